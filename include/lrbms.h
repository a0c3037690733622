/*
 * lrbms.h -- C ABI of the MI355X (gfx950) library for the online step of the
 * Localized Reduced Basis Multiscale (LRBMS) method for two-phase flow
 * (Kaulmann, Flemisch, Haasdonk, Lie, Ohlberger, arXiv:1405.2810).
 *
 * One online step (Alg. 3, step 5) is
 *     lrbms_online_assemble   a) mobility of s^n and the reduced system
 *     lrbms_online_solve      a) reduced SPD solve  A_N p_N = f_N
 *     lrbms_reconstruct_flux  b)+c) p_h = Phi p_N and one normal flux per face
 *     lrbms_transport_step    d) DG upwind explicit Euler saturation + limiter
 *
 * Conventions (all arrays are plain C arrays; "device" = HIP device memory):
 *  - cells c = i + nx*(j + ny*k), x fastest; nz = 1 in 2D.
 *  - faces: all x-faces, then y-faces, then z-faces.  The x-face (i,j,k),
 *    i in [0,nx], is i + (nx+1)*(j + ny*k); y-faces i + nx*(j + (ny+1)*k);
 *    z-faces i + nx*(j + ny*k).  Fluxes are oriented along +axis.
 *  - P1 fields (saturation, pressure, mobility fields) are stored SoA in the
 *    L2-orthonormal cell basis phi_0 = |e|^-1/2, phi_{a+1} = sqrt(3) xi_a
 *    |e|^-1/2 (xi_a in [-1,1] the local coordinate): coefficient k of cell c
 *    at index k*ncell + c, r = dim+1 coefficients per cell.
 *  - coarse boxes E are numbered lexicographically (x fastest) from the cut
 *    indices; inside a box cells are listed x fastest.  A local basis
 *    Phi^E is stored as N_E consecutive functions, each an (r, n_E) array
 *    (coefficient-major); boxes are concatenated in box order.
 *  - p_N: box blocks in box order, each of length N_E.
 *  - Return codes: 0 success, negative errors (LRBMS_E_*), positive warnings.
 *    Errors found on the device (a non-positive pivot, a non-finite residual,
 *    flux or saturation) and the CFL warning of a transport step set the
 *    model's status words; lrbms_model_status returns them, and so does
 *    every online call while checks are on (lrbms_model_set_checks).  The
 *    online calls are asynchronous otherwise.  No C++ exception crosses the
 *    ABI.
 *    lrbms_last_error() gives a thread-local message for the last error.
 *  - Every call taking a `stream` (a hipStream_t, 0 = null stream) enqueues
 *    work asynchronously on it and does not synchronize unless stated.
 *  - Ownership: the library copies the problem description and the bases at
 *    creation and owns everything inside a model; caller buffers (s, p_N,
 *    fluxes, p_h, flags) are never freed or retained by the library.
 */
#ifndef LRBMS_H
#define LRBMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LRBMS_OK = 0,
  LRBMS_E_ARG = -1,        /* invalid argument (checked synchronously)          */
  LRBMS_E_STATE = -2,      /* call order violated (e.g. solve before assemble)  */
  LRBMS_E_OOM = -3,        /* device or host allocation failed                   */
  LRBMS_E_HIP = -4,        /* a HIP runtime call failed                          */
  LRBMS_E_NOT_SPD = -5,    /* non-positive pivot in the reduced Cholesky         */
  LRBMS_E_NONFINITE = -6,  /* NaN/Inf detected                                   */
  LRBMS_E_ADMIT = -7,      /* serving: request exceeds the memory budget         */
  LRBMS_W_CFL = 1          /* warning: the time step exceeds the CFL estimate    */
};

/* Reduced assembly modes.
 * DIRECT:     A_N = Phi^T A(lambda(s)) Phi, f_N = Phi^T l(lambda(s)), i.e. the
 *             Galerkin projection of the SWIP forms (Sec. 3.2 eq. swipBilP and the
 *             linear form l_h) onto W_N (Def. coarseScalePressure) with the exact
 *             mobility, 2-point Gauss rules on cells and faces.
 * DIRECT_FIT: the same with gamma = sum_q theta_q Lambda^q, theta from the
 *             least-squares fit (eq. leastSquaresFit).
 * AFFINE:     A_N = c + sum_q theta_q b_q, f_N = e + sum_q theta_q d_q
 *             (Sec. 4.4 eq. reducedSystem); needs mobility profiles.          */
enum { LRBMS_DIRECT = 0, LRBMS_DIRECT_FIT = 1, LRBMS_AFFINE = 2 };

enum { LRBMS_BC_INTERIOR = 0, LRBMS_BC_NEUMANN = 1, LRBMS_BC_DIRICHLET = 2 };

/* Problem statement (Sec. 2 and Sec. 3.1 of the paper).  The densities and
 * the gravity vector are part of the statement; this library solves the
 * case without gravity (the paper's experiments have none), so a non-zero
 * grav is rejected with LRBMS_E_ARG and the densities are not used.
 * All pointers are HOST pointers and are copied by the create calls.        */
typedef struct lrbms_problem {
  int32_t dim;              /* 2 or 3                                               */
  int32_t n[3];             /* fine cells per axis (n[2] = 1 in 2D)                 */
  double len[3];            /* domain lengths (len[2] ignored in 2D)                */
  int32_t nc[3];            /* coarse boxes per axis (nc[2] = 1 in 2D)              */
  const int32_t* cuts[3];   /* nc[a]+1 increasing cut indices per axis, 0 .. n[a]   */
  const double* perm;       /* [ncell] scalar permeability kappa                    */
  const double* poro;       /* [ncell] porosity phi                                 */
  double visc_w, visc_o;    /* viscosities eta_w, eta_o (eq. brooksCorey)           */
  int32_t relperm;          /* 0: k_rw = s, k_ro = 1-s; 1: k_rw = s^cw, k_ro = (1-s)^co
                               (s clipped to [0,1] inside the laws)                 */
  double corey_w, corey_o;
  const int8_t* bc_type;    /* [nface] LRBMS_BC_*                                   */
  const double* bc_val;     /* [nface] Neumann outward flux density v_N / Dirichlet p_D */
  const int8_t* bc_sat;     /* [nface] 1 on saturation Dirichlet (inflow) faces     */
  const double* bc_sval;    /* [nface] s_D                                          */
  const double* q1;         /* [ncell] pressure source density                      */
  const double* q2;         /* [ncell] saturation source density                    */
  double penalty_c;         /* c_f; sigma_f = c_f / max(eta) * 2 a1 a2/(a1+a2)      */
  int32_t weights;          /* 0: SWIP mean weights a2/(a1+a2); 1: literal a1/(a1+a2) */
  double sat_penalty_scale; /* multiplies sigma_f in the saturation equation        */
  int32_t limiter;          /* 1: apply the slope limiter after each Euler step     */
  double dt;                /* time step (> 0)                                      */
  double dens_w, dens_o;    /* densities rho_w, rho_o (finite; unused without gravity) */
  double grav[3];           /* gravity vector G; must be zero                       */
} lrbms_problem;

typedef struct lrbms_model lrbms_model;

/* Sizes of a model (host query, no device work). */
typedef struct lrbms_model_info {
  int32_t dim, r, ncell, nface, n_sub, n_iface, N, n_profiles;
  int64_t n_block_entries;  /* doubles in the block storage of A_N                 */
  int64_t device_bytes;     /* device memory held by the model                      */
} lrbms_model_info;

/* Offline options for lrbms_build_offline_bases (Alg. 2 without the greedy
 * selection: time-of-flight profiles, training snapshots, local Gram-Schmidt
 * with an optional cap).                                                       */
typedef struct lrbms_offline_opts {
  int32_t M;                /* number of mobility profiles (3 .. 64)                */
  int32_t n_train;          /* training parameters: rows of the mu array            */
  int32_t ne_cap;           /* maximum local basis size N_E (1 .. 63)               */
  int32_t unit_functions;   /* 1: put 1_E first in every local basis                */
  double horizon;           /* T of the profile thresholds (q-1) T/(M-2), > 0       */
  double pcg_rtol;          /* relative residual of the fine solves (> 0)           */
  int32_t pcg_maxit;        /* CG iteration limit per fine solve (> 0)              */
  double tof_tol;           /* relative change that ends the time-of-flight sweeps  */
  int32_t tof_maxit;        /* sweep limit (> 0)                                    */
  int32_t keep_profiles;    /* 1: keep the linearly independent profiles (AFFINE,
                               DIRECT_FIT); 0: a model without profiles             */
  const double* d_s0;       /* device [r*ncell] saturation whose flow defines the time
                               of flight (re-basing from a later state); NULL: s = 0 */
  int32_t basis_method;     /* LRBMS_BASIS_GS or LRBMS_BASIS_PCA (local bases below) */
  double pca_eps;           /* PCA: discarded energy <= pca_eps^2 of the total (>= 0) */
} lrbms_offline_opts;

/* Local bases from snapshots, in every box on the device (one workgroup per
 * box), 1_E first when unit functions are asked for, at most ne_cap functions:
 *  LRBMS_BASIS_GS:  the restrictions of the snapshots in order, Gram-Schmidt
 *                   in L2(E) (two passes, rejection of remaining norms
 *                   <= 1e-8 of the original) (Alg. 2 step 2e);
 *  LRBMS_BASIS_PCA: the method of snapshots (Alg. 2 step 3): the restrictions
 *                   with their components along 1_E removed, the eigenpairs
 *                   of their Gram matrix (Jacobi rotations), the fewest
 *                   leading modes whose discarded eigenvalues sum to at most
 *                   pca_eps^2 of the total, each added by the Gram-Schmidt
 *                   step above; at most 64 snapshots.                         */
enum { LRBMS_BASIS_GS = 0, LRBMS_BASIS_PCA = 1 };

/* What the offline stage did (filled when the caller passes a non-NULL pointer). */
typedef struct lrbms_offline_report {
  int32_t n_solves;         /* fine solves: the initial pressure + n_train snapshots */
  int32_t pcg_iters_max;    /* largest CG iteration count of one solve              */
  int64_t pcg_iters_total;
  double pcg_relres_max;    /* largest final relative residual                      */
  int32_t tof_sweeps;       /* block-Jacobi sweeps of the time of flight            */
  int32_t n_profiles_kept;  /* profiles kept in the model                           */
} lrbms_offline_report;

/* Create a model from given local bases (parity runs use this).
 *  basis_sizes: host [n_sub] N_E per box (1 .. 63)
 *  basis:       host, concatenated per-box arrays (N_E, r, n_E) as documented
 *  n_profiles/profiles: host [n_profiles][r*ncell] total-mobility profiles for
 *               AFFINE / DIRECT_FIT (linearly independent; n_profiles may be 0)
 * The model precomputes the affine terms when profiles are given.  The
 * reduced solver's plan of a new model takes the leaf size with the shortest
 * launch sequence (2, 4 or 8 boxes), splits panel steps of at least
 * LRBMS_STEP_SPLIT_MIN tiles (environment, default 1024) and the backward
 * product of fronts with m u >= LRBMS_BW_SPLIT_MIN (default 2^14);
 * lrbms_model_autotune replaces these shapes by measured ones.
 * Errors: LRBMS_E_ARG for inconsistent sizes, LRBMS_E_OOM, LRBMS_E_HIP.       */
int lrbms_model_create(const lrbms_problem* prob, const int32_t* basis_sizes,
                       const double* basis, int32_t n_profiles, const double* profiles,
                       lrbms_model** out);

/* Create a model whose local bases come from global snapshots (host,
 * [n_snap][r*ncell], copied to the device once): local bases by
 * basis_method (LRBMS_BASIS_GS or LRBMS_BASIS_PCA with pca_eps, as
 * described above), 1_E first when unit_functions is set, at most ne_cap
 * functions per box.  Profiles as in lrbms_model_create.  LRBMS_E_ARG also
 * when a box ends with an empty local basis.                                 */
int lrbms_model_create_from_snapshots(const lrbms_problem* prob, int32_t n_snap,
                                      const double* snapshots, int32_t ne_cap,
                                      int32_t unit_functions, int32_t basis_method,
                                      double pca_eps, int32_t n_profiles,
                                      const double* profiles, lrbms_model** out);

/* Fine pressure of Def. pressureDG (the SWIP discretisation on the fine grid,
 * b_h(p_h, v; gamma) = l_h(v; gamma)) solved on the device by conjugate
 * gradients preconditioned with one multigrid V-cycle (below), x0 = 0.  Also
 * the fine reference of the online step and the snapshot solver of the
 * offline stage.
 *  d_field: device [r*ncell]; with kind LRBMS_FIELD_SATURATION the mobility is
 *           lambda(s) of this saturation, with LRBMS_FIELD_MOBILITY it is the
 *           field itself (a P1 field, e.g. a training mobility of Alg. 2)
 *  d_p:     device [r*ncell], receives p_h
 *  iterations, relres: host outputs (nullable): CG iterations and the final
 *           relative residual |l - A p| / |l|, from the recursion
 * Synchronous (default stream); allocates its work arrays per call.
 * The preconditioner is one symmetric multigrid V-cycle: damped cell-block
 * Jacobi on P1, then the cell-wise constants, whose Galerkin operator is the
 * mobility-free penalty part, coarsened by aggregation down to a dense solve.
 * Errors: LRBMS_E_ARG, LRBMS_E_OOM, LRBMS_E_HIP, LRBMS_E_NOT_SPD (a singular
 * cell block, a non-positive curvature or an indefinite preconditioner),
 * LRBMS_E_NONFINITE, LRBMS_E_STATE when maxit iterations end above rtol
 * (d_p then holds the last iterate).                                         */
enum { LRBMS_FIELD_SATURATION = 0, LRBMS_FIELD_MOBILITY = 1 };
int lrbms_fine_pressure(const lrbms_problem* prob, const double* d_field, int32_t kind,
                        double rtol, int32_t maxit, double* d_p, int32_t* iterations,
                        double* relres);

/* Time of flight of eq. timeOfFlight (Sec. 3.6) for the face fluxes d_flux
 * (device, [nface], oriented along +axis, e.g. from lrbms_reconstruct_flux):
 * upwind DG P1, the own trace on outflow faces, the neighbour trace on inflow
 * faces and zero on inflow boundary faces; right-hand side the porosity.
 * Solved by block-Jacobi sweeps (each cell solves its r x r block with the
 * upwind traces of the previous sweep), exact after as many sweeps as the
 * longest upwind chain has cells when the flow has no cycles; stops when the
 * largest coefficient change is <= tol times the largest coefficient.
 *  d_tau: device [r*ncell], receives tau;  sweeps: host output (nullable)
 * Synchronous (default stream).  Errors: LRBMS_E_ARG, LRBMS_E_OOM, LRBMS_E_HIP,
 * LRBMS_E_NOT_SPD (a cell block is singular, e.g. a cell with no flux at
 * all), LRBMS_E_NONFINITE, LRBMS_E_STATE when maxit sweeps end unconverged. */
int lrbms_time_of_flight(const lrbms_problem* prob, const double* d_flux, double tol,
                         int32_t maxit, double* d_tau, int32_t* sweeps);

/* lrbms_time_of_flight for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operation, arguments, results and errors, but every
 * work buffer (the cell and face blocks, the sweep vector, the partial
 * maxima, the porosity and the status word) lives in one fixed scratch
 * array of 128 MiB per device inside the library, held until the process
 * ends; no hipMalloc, hipFree or allocating library call is made.  The
 * problem must fit that array: (1 + ncell + r^2 ncell + 2 dim r^2 ncell +
 * 2 r ncell + 2 ceil(ncell/256) + 2) doubles (up to about 320,000 cells in
 * 2D and 138,000 in 3D); LRBMS_E_ARG otherwise.  Calls on one device share the array: calls
 * that overlap in time on the same device race and must be serialized by the
 * caller; every call clears what it needs at its start.                     */
int lrbms_time_of_flight_noalloc(const lrbms_problem* prob, const double* d_flux, double tol,
                                 int32_t maxit, double* d_tau, int32_t* sweeps);

/* Greedy basis construction (Alg. 2 step 2, the error-driven extension) on the
 * device, with the true error measure: the energy norm |p_H(mu) - p_h(mu)| of
 * b_h(., .; sum_q mubar_q Lambda^q).  Steps 1a-1c as lrbms_build_offline_bases
 * (options M, n_train, horizon, solver tolerances, d_s0, keep_profiles; ne_cap
 * and unit_functions are not used).  Then the fine snapshots of all n_train
 * training parameters are computed as one batch and kept on the device; each
 * iteration solves, for every training parameter, the reduced system of the
 * current local bases (affine terms with theta = mu), measures the error,
 * picks the worst parameter (first of equal maxima) and extends every local
 * basis by Gram-Schmidt with its snapshot.  Starts from empty local bases;
 * stops when the largest error is <= tol, the total size reaches n_max, no
 * basis grows, or after 63 extensions.
 *  mu:      host [n_train][M];  mu_bar: host [M] or NULL (1/M each)
 *  chosen:  host [max_iter] (nullable): the parameter added in each extension
 *  errors:  host [max_iter] (nullable): the largest error of each evaluation
 *  n_iter:  host (nullable): number of evaluations (extensions + 1 at most)
 * Synchronous.  Errors: as lrbms_build_offline_bases; LRBMS_E_ARG when a box
 * ends with no basis function.                                                 */
int lrbms_build_greedy_bases(const lrbms_problem* prob, const lrbms_offline_opts* opts,
                             const double* mu, int32_t n_max, double tol, const double* mu_bar,
                             lrbms_model** out, int32_t* chosen, double* errors,
                             int32_t max_iter, int32_t* n_iter, lrbms_offline_report* report);

/* Fine reference: the high-dimensional IMPES scheme of Alg. 1 on the device
 * (the accuracy reference that the LRBMS online step replaces).  A handle owns
 * the problem on the device and the fine solver's work arrays and coarse
 * hierarchy.  One lrbms_fine_step is one time step: p_h from lambda(d_sat)
 * (lrbms_fine_pressure's solver; warm != 0 starts CG from the contents of
 * d_ph, e.g. the previous step's pressure), the face fluxes of Def.
 * velocityDG, the saturation step of Def. saturationDG and the limiter as in
 * lrbms_transport_step.
 *  d_sat (in), d_ph (in/out), d_flux, d_sat_out, d_flags (nullable): device
 *  arrays as in the online calls; d_sat_out must not alias d_sat.
 *  iterations, relres: host outputs (nullable).
 * Synchronous (default stream).  Errors as lrbms_fine_pressure.               */
typedef struct lrbms_fine lrbms_fine;
int lrbms_fine_create(const lrbms_problem* prob, lrbms_fine** out);
int lrbms_fine_step(lrbms_fine* f, const double* d_sat, double rtol, int32_t maxit, int32_t warm,
                    double* d_ph, double* d_flux, double* d_sat_out, uint8_t* d_flags,
                    int32_t* iterations, double* relres);
void lrbms_fine_destroy(lrbms_fine* f);

/* Offline stage on the device (Alg. 2 steps 1-2 without the error-driven
 * selection): initial pressure at s0 (default 0) by lrbms_fine_pressure, its face
 * fluxes (Def. velocityDG), the time of flight, the M profiles of Alg. 2
 * step 1c (Lambda^1 = lambda(0), Lambda^M = lambda(1), Lambda^q = lambda(0)
 * where the cell mean of tau exceeds (q-1) T/(M-2), else lambda(1)), one
 * fine snapshot per training mobility gamma = sum_q mu_q Lambda^q (in row
 * order, kept on the device), then the local bases by opts->basis_method.
 * With keep_profiles the model keeps the profiles that are linearly
 * independent of the ones before them (in q order; Gram-Schmidt with a
 * relative threshold of 1e-12).
 *  mu:     host [n_train][M] training parameters
 *  report: host output (nullable)
 * Untimed setup, synchronous; the bases can be read back with
 * lrbms_model_export_basis and the profiles with lrbms_model_export_profiles.
 * Errors: those of lrbms_fine_pressure and lrbms_time_of_flight, and
 * LRBMS_E_ARG when a box ends with an empty local basis.                     */
int lrbms_build_offline_bases(const lrbms_problem* prob, const lrbms_offline_opts* opts,
                              const double* mu, lrbms_model** out,
                              lrbms_offline_report* report);

int lrbms_model_get_info(const lrbms_model* m, lrbms_model_info* info);

/* Copy the bases (host): sizes [n_sub], basis as in lrbms_model_create.       */
int lrbms_model_export_basis(const lrbms_model* m, int32_t* sizes, double* basis);

/* Copy the model's mobility profiles (host, [n_profiles][r*ncell]).           */
int lrbms_model_export_profiles(const lrbms_model* m, double* profiles);

/* a) Mobility of d_sat (device, [r*ncell]) and the reduced system A_N, f_N
 *    (kept inside the model in block storage).  mode: LRBMS_DIRECT / _FIT / AFFINE. */
int lrbms_online_assemble(lrbms_model* m, const double* d_sat, int32_t mode, void* stream);

/* a) Factor A_N (multifrontal block Cholesky, nested-dissection order over the
 *    coarse boxes) and solve A_N p_N = f_N (eq. reducedSystem); d_pN (device,
 *    [N]) receives p_N.  Then the model's refinement steps (default 1): the
 *    residual f_N - A_N p_N in double-double arithmetic, a forward and a
 *    backward substitution of it with the stored factor, p_N += correction.
 *    LRBMS_E_STATE if no assembly preceded (synchronous).  Device-detected:
 *    a non-positive pivot sets LRBMS_E_NOT_SPD, a non-finite residual
 *    LRBMS_E_NONFINITE in the status word (lrbms_model_status).              */
int lrbms_online_solve(lrbms_model* m, double* d_pN, void* stream);

/* Iterative refinement steps of every later reduced solve of the model
 * (0..4; 1 at creation).  LRBMS_E_ARG outside 0..4; LRBMS_E_STATE while a
 * batch or server holds the model (the members of a batch must agree).    */
int lrbms_model_set_refinement(lrbms_model* m, int32_t steps);

/* b)+c) p_h = Phi p_N and the face fluxes of Def. velocityDG with lambda(d_sat):
 *    d_flux (device, [nface]) along +axis; on Neumann faces the flux is v_N |f|.
 *    d_ph (device, [r*ncell]) receives p_h when non-NULL.                     */
int lrbms_reconstruct_flux(lrbms_model* m, const double* d_pN, const double* d_sat,
                           double* d_flux, double* d_ph, void* stream);

/* d) Explicit Euler DG upwind saturation step (Def. saturationDG) and, if the
 *    problem enables it, the slope limiter (eq. limiterMain).  d_sat_out must
 *    not alias d_sat.  d_flags (device, [ncell], nullable) receives 1 on
 *    limited cells.                                                             */
int lrbms_transport_step(lrbms_model* m, const double* d_sat, const double* d_flux,
                         double* d_sat_out, uint8_t* d_flags, void* stream);

/* Copy the reduced system of the last assembly: blocks (host, n_block_entries
 * doubles: diagonal blocks N_E x N_E row-major in box order, then one
 * coupling block A[E_lo][E_hi] (N_lo x N_hi, row-major) per coarse interface)
 * and f_N (host, [N]).  Synchronizes the model's last stream.                  */
int lrbms_copy_reduced_system(lrbms_model* m, double* blocks, double* fN);

/* Coarse interfaces (host): for interface t, axis[t], lo[t], hi[t] box numbers. */
int lrbms_model_interfaces(const lrbms_model* m, int32_t* axis, int32_t* lo, int32_t* hi);

/* Least-squares coefficients theta of the last AFFINE / DIRECT_FIT assembly
 * (host, [n_profiles]).  Synchronizes.                                          */
int lrbms_copy_theta(lrbms_model* m, double* theta);

/* Host-only inspection of the reduced solver's symbolic analysis (no device
 * work): the nested-dissection assembly tree, fronts, index maps and the
 * per-level work lists that the numeric kernels execute, including the split
 * backward products (environment variable LRBMS_BW_SPLIT_MIN, as for a
 * model), flattened into int64 records (layout documented in the Python
 * binding).  With buf == NULL
 * or cap too small only *needed is set.  leaf_max: largest region (in boxes)
 * that becomes a leaf front.                                                   */
int lrbms_solver_plan_export(const lrbms_problem* prob, const int32_t* basis_sizes,
                             int32_t leaf_max, int64_t* buf, int64_t cap, int64_t* needed);

/* The same for the combined plan of a fused batch of n problems (member k
 * with basis sizes basis_sizes[k] and leaf size leaf_max[k]): fronts, nodes
 * and work lists of all members, level by level, with their offsets into
 * shared storage (A_N blocks, f_N and p_N of the members one after another,
 * in member order).  Host only; LRBMS_E_ARG also when an offset of the plan
 * would fall outside its storage.                                              */
int lrbms_solver_plan_export_batch(const lrbms_problem* const* probs,
                                   const int32_t* const* basis_sizes, const int32_t* leaf_max,
                                   int32_t n, int64_t* buf, int64_t cap, int64_t* needed);

/* Autotuner of the box assembly and of the reduced solver's shapes.  First
 * both box-assembly variants (lrbms_model_set_assembly_variant) are timed on
 * reps DIRECT assemblies of d_sat and the faster is kept.  Then the solver: the leaf size of the nested
 * dissection (1, 2, 4, 8 or 16 boxes) and the smallest panel step that is
 * split in two launches (256 or 1024 tiles, or never); then, on the fastest
 * of those, the smallest front (m u entries of L_US: 2^12, 2^14, 2^16, 2^18
 * or never) whose backward product is split over many workgroups.
 * Assembles the reduced system of d_sat (device, [r*ncell]; DIRECT), then for
 * every candidate builds the solver plan, times reps solves (after two
 * untimed ones) with HIP events on the default stream, and keeps the fastest
 * plan in the model.  Then it measures the error of the unrefined reduced
 * solve on that system (the relative size of one refinement step's
 * correction) and sets the model's refinement steps to 0 when it is below
 * 1e-13, else keeps them (at least 1).  The report (nullable) gives the
 * chosen shapes, its time per solve, the time of the plan the model had
 * before, the number of candidates timed, the measured unrefined error and
 * the refinement steps kept.  Synchronous; allocates; results of later
 * solves differ from before only by rounding (another elimination order, or
 * no refinement step).
 * LRBMS_E_STATE while the model belongs to a batch or server.                 */
typedef struct lrbms_tune_report {
  int32_t leaf_max, split_min;   /* split_min: 0 = never split */
  int32_t n_candidates, bw_split_min;   /* bw_split_min: 0 = never split */
  double us_per_solve, us_before;
  /* error of the unrefined solve, measured as |p_1 - p_0| / |p_1| for the
   * solutions without (p_0) and with one refinement step (p_1) on the tuning
   * state; the model keeps its refinement steps unless this is below 1e-13
   * (three orders under the 1e-10 parity bound), then it solves unrefined  */
  double unrefined_error;
  int32_t refine;
  int32_t asm_variant;   /* box assembly variant kept (lrbms_model_set_assembly_variant) */
  double asm_us[2];      /* time of one DIRECT assembly with variant 0 and with 1      */
} lrbms_tune_report;
int lrbms_model_autotune(lrbms_model* m, const double* d_sat, int32_t reps,
                         lrbms_tune_report* report);

/* Installs the reduced solver's plan for given shapes (the fields of a tune
 * report: leaf_max 1..64 boxes, split_min 0 = never split else >= 1 tile,
 * bw_split_min 0 = never split else >= 1 entry), as the autotuner would
 * after choosing them: for reusing a tuned configuration without timing
 * it again.  Synchronous; allocates.  LRBMS_E_ARG for shapes out of range
 * or a plan that does not fit its storage, LRBMS_E_STATE while the model
 * belongs to a batch or server, LRBMS_E_OOM.                                 */
int lrbms_model_set_solver_shapes(lrbms_model* m, int32_t leaf_max, int32_t split_min,
                                  int32_t bw_split_min);

/* Box assembly variant of the model (Def. coarseScalePressure, the diagonal
 * blocks Phi_E^T A_E Phi_E): 0 = four waves per workgroup, each thread
 * forming K Phi for several columns of one cell (chunks of 32 cells in 3D
 * up to 47 basis functions, else 64); 1 = six waves, one (cell, column) item
 * per thread with all neighbour loads in flight at once (chunks of 30 cells
 * in 3D, 64 in 2D).  Same arithmetic per entry; the chunk partials, and so
 * the rounding of A_N, differ.  Synchronous.  LRBMS_E_ARG for another
 * variant, LRBMS_E_STATE while the model belongs to a batch or server.       */
int lrbms_model_set_assembly_variant(lrbms_model* m, int32_t variant);

/* Kernel timing, for roofline measurement (off by default).
 * lrbms_profile_enable synchronizes the model's last stream, clears the
 * counters and switches timing on (enable != 0) or off.  While on, every
 * kernel launched by the four online calls is bracketed by a pair of HIP
 * events on the call's stream (a few microseconds of added gap per launch).
 * lrbms_profile_read waits for the recorded events and fills up to cap
 * entries, one per kernel kind that ran: launches, summed device time, and
 * the algorithmic flops and bytes of those launches (the arithmetic of what
 * the kernel computes and the data it must read and write once, 8 B per
 * double, from the model's sizes); *n_out = number of kinds that ran.       */
typedef struct lrbms_kernel_stat {
  char name[40];
  int64_t launches;
  double total_ms;
  double flops;
  double bytes;
} lrbms_kernel_stat;
int lrbms_profile_enable(lrbms_model* m, int32_t enable);
int lrbms_profile_read(lrbms_model* m, lrbms_kernel_stat* out, int32_t cap, int32_t* n_out);

/* ---- many simulations on one device ------------------------------------------
 * Both patterns run, for each simulation, exactly the four online calls above
 * (one time step of Alg. 3 step 5: assembly in the given mode, reduced solve,
 * flux reconstruction, transport + limiter) and copy the new state over the
 * simulation's state buffer, so each simulation's result equals that of the
 * plain per-simulation path, bit for bit.  A model may belong to one batch or
 * server at a time and must not be stepped elsewhere meanwhile; destroy the
 * batch or server (or detach) before destroying its models (a member of a
 * fused batch or of a server refuses to be destroyed until then).  Not thread-safe:
 * one host thread drives a batch or server.  Kernel timing
 * (lrbms_profile_enable) must be off for its models (LRBMS_E_STATE otherwise). */

typedef struct lrbms_batch lrbms_batch;
#define LRBMS_BATCH_GRAPH 1        /* capture the whole batched step into one HIP graph */
#define LRBMS_BATCH_FUSED_SOLVE 2  /* one reduced solve for all members (shared launches) */

/* Batched ensemble: n models (distinct) advanced together.  The batch owns,
 * per simulation, p_N [N], the face fluxes [nface] and the next state
 * [r*ncell] (device).  mode: LRBMS_DIRECT / _FIT / AFFINE, available for
 * every model (LRBMS_E_ARG otherwise).  flags: LRBMS_BATCH_GRAPH and/or
 * LRBMS_BATCH_FUSED_SOLVE.  Fused: the members' reduced systems are solved
 * together: one multifrontal plan holds the fronts of every member (level by
 * level), so each launch of the solver processes the fronts of all members
 * at that point of their schedules; the members' A_N and f_N live in storage
 * of the batch while it exists (a model belongs to at most one fused batch).
 * Members may differ in refinement steps: each takes its own (a member is
 * masked off the fused refinement steps beyond its count).
 * Errors: LRBMS_E_ARG, LRBMS_E_OOM, LRBMS_E_HIP.                              */
int lrbms_batch_create(lrbms_model* const* models, int32_t n, int32_t mode, int32_t flags,
                       lrbms_batch** out);

/* One time step of every simulation of the batch, asynchronous on `stream`:
 * d_sat[i] (device, [r*ncell] of model i) is advanced in place; d_flags
 * (nullable; else an array of n nullable device pointers, [ncell] each)
 * receives the limiter flags.  Every simulation runs on a branch of its own
 * (up to 64 branches, then round robin), forked from and joined back into
 * `stream`.  With LRBMS_BATCH_GRAPH the branches are captured once into a
 * HIP graph (recaptured when the state or flag pointers change) and every
 * step is one graph launch; otherwise the branches are launched directly.
 * Errors: LRBMS_E_ARG, LRBMS_E_STATE, LRBMS_E_HIP.                             */
int lrbms_batch_step(lrbms_batch* b, double* const* d_sat, uint8_t* const* d_flags, void* stream);

/* Synchronize the device; the first non-zero status of the fused solve or of
 * the members (as lrbms_model_status), else 0.                                */
int lrbms_batch_status(lrbms_batch* b);

/* Device pointers of simulation i's p_N and face fluxes of the last step.  */
int lrbms_batch_buffers(lrbms_batch* b, int32_t i, double** d_pN, double** d_flux);
void lrbms_batch_destroy(lrbms_batch* b);

/* Serving loop with continuous batching.  Simulations are attached with
 * their state buffer and admitted, in attach order, while the sum of the
 * admitted simulations' footprints (the model's device bytes plus the step
 * buffers the server allocates on admission: p_N, fluxes, next state) stays
 * within hbm_budget bytes.  A request is one time step of one simulation.
 * Requests are dispatched in submit order onto up to max_slots (1..64) slot
 * streams, at most one request per simulation in flight (its steps are
 * sequential); requests of simulations not yet admitted, or whose previous
 * step still runs, wait while later ones go ahead.  The server makes
 * progress (retires finished requests, admits, dispatches) inside attach,
 * submit, poll, detach and drain; a serving loop calls poll regularly.
 * Latency of a request = host time from its submit to the poll or drain
 * that first sees it finished.                                                */
typedef struct lrbms_server lrbms_server;
typedef struct lrbms_server_info_t {
  int64_t resident_bytes, budget_bytes;
  int32_t n_pending, n_in_flight, n_admitted, n_waiting;
} lrbms_server_info_t;

/* Errors: LRBMS_E_ARG (budget <= 0, max_slots outside 1..64, unknown mode),
 * LRBMS_E_HIP.                                                                 */
int lrbms_server_create(int64_t hbm_budget, int32_t max_slots, int32_t mode, lrbms_server** out);

/* Attach model m with its state d_sat (device, [r*ncell], advanced in place by
 * every request; the device is synchronized first, so work that wrote it on
 * any stream is complete); *sim_id receives the simulation's id.  LRBMS_E_ADMIT when
 * the footprint alone exceeds the budget, LRBMS_E_ARG when m is attached
 * already or lacks the server's mode.  A simulation that does not fit yet
 * waits for others to be detached.                                            */
int lrbms_server_attach(lrbms_server* s, lrbms_model* m, double* d_sat, int32_t* sim_id);

/* Queue one time step of simulation sim_id under the caller's request id.  */
int lrbms_server_submit(lrbms_server* s, int32_t sim_id, uint64_t req_id);

/* Copy up to cap finished requests (oldest first): ids, latency in ms
 * (nullable) and status (nullable; 0 or a negative LRBMS_E_* of a launch).
 * Device-detected errors are read with lrbms_model_status.                    */
int lrbms_server_poll(lrbms_server* s, uint64_t* req_ids, double* latency_ms, int32_t* status,
                      int32_t cap, int32_t* n_done);

/* Progress until no request is queued or in flight.  LRBMS_E_ADMIT when the
 * remaining requests belong to simulations that cannot be admitted until
 * others are detached.                                                        */
int lrbms_server_drain(lrbms_server* s);

/* Detach a simulation (waits for its request in flight; LRBMS_E_STATE while it
 * has queued requests), free its step buffers and admit waiting ones.       */
int lrbms_server_detach(lrbms_server* s, int32_t sim_id);
int lrbms_server_info(const lrbms_server* s, lrbms_server_info_t* info);
/* Fused dispatch (call before the first attach; on != 0): the pending
 * requests of distinct admitted simulations, up to max_slots, form a wave:
 * their assemblies run on the slot streams, then ONE reduced solve by the
 * combined multifrontal plan of every admitted simulation runs with the
 * wave's members active and the others masked off (their workgroups return
 * at once), then their fluxes and transport run on the slot streams.  One
 * wave is on the device at a time; requests arriving meanwhile join the
 * next one (continuous batching).  The combined plan and storage (A_N, f_N,
 * p_N of every member) are rebuilt whenever the admitted set changes.  A
 * wave takes the largest refinement steps of its members, each member only
 * its own.  Each simulation's result is the one its plain path gives, bit
 * for bit.
 * LRBMS_E_STATE after the first attach.                                      */
int lrbms_server_set_fused(lrbms_server* s, int32_t on);
void lrbms_server_destroy(lrbms_server* s);

/* Synchronize with the model's last stream and return its device status:
 * the first error (LRBMS_E_NOT_SPD: non-positive pivot; LRBMS_E_NONFINITE:
 * NaN/Inf in the reduced residual, a face flux or the new saturation), else
 * LRBMS_W_CFL if a transport step's CFL number, dt max|f_w'| times a cell's
 * outflow over phi |e| (Def. saturationDG, explicit Euler), exceeded 1/2,
 * else 0.  The words keep their value (reading does not clear them).       */
int lrbms_model_status(lrbms_model* m);

/* on != 0: every online call (assemble, solve, reconstruct_flux,
 * transport_step) synchronizes its stream and returns lrbms_model_status
 * (for callers that want errors and the CFL warning at the call that
 * caused them); 0 (the default): the calls stay asynchronous.  LRBMS_E_ARG
 * for a NULL model.                                                         */
int lrbms_model_set_checks(lrbms_model* m, int32_t on);

const char* lrbms_last_error(void);
/* Frees the model.  A model that belongs to a fused batch or is attached to a
 * server is not destroyed (lrbms_last_error says why): destroy the batch or
 * the server, or detach it, first.                                             */
void lrbms_model_destroy(lrbms_model* m);

#ifdef __cplusplus
}
#endif
#endif /* LRBMS_H */
