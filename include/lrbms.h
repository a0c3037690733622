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
 *    Errors found on the device set the model's status word; the next call
 *    or lrbms_model_status returns them.  No C++ exception crosses the ABI.
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

/* Problem statement (Sec. 2 and Sec. 3.1 of the paper; gravity is zero).
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
} lrbms_problem;

typedef struct lrbms_model lrbms_model;

/* Sizes of a model (host query, no device work). */
typedef struct lrbms_model_info {
  int32_t dim, r, ncell, nface, n_sub, n_iface, N, n_profiles;
  int64_t n_block_entries;  /* doubles in the block storage of A_N                 */
  int64_t device_bytes;     /* device memory held by the model                      */
} lrbms_model_info;

/* Offline options for lrbms_build_offline_bases (Alg. 2 without the greedy loop:
 * TOF profiles, training snapshots, local Gram-Schmidt, optional cap).         */
typedef struct lrbms_offline_opts {
  int32_t M;                /* number of mobility profiles (>= 3)                   */
  int32_t n_train;          /* training snapshots: the M profiles, then seeded mixes */
  int32_t ne_cap;           /* maximum local basis size N_E (<= 63)                 */
  int32_t unit_functions;   /* 1: put 1_E first in every local basis                */
  int32_t n_steps;          /* N_T, the profiles use T = N_T * dt                   */
  uint64_t seed;            /* seed of the training mixes                           */
  double pcg_rtol;          /* relative residual of the fine snapshot solves        */
  int32_t pcg_maxit;
  int32_t keep_profiles;    /* 1: keep the (deduplicated) profiles for AFFINE       */
} lrbms_offline_opts;

/* Create a model from given local bases (parity runs use this).
 *  basis_sizes: host [n_sub] N_E per box (1 .. 63)
 *  basis:       host, concatenated per-box arrays (N_E, r, n_E) as documented
 *  n_profiles/profiles: host [n_profiles][r*ncell] total-mobility profiles for
 *               AFFINE / DIRECT_FIT (linearly independent; n_profiles may be 0)
 * The model precomputes the affine terms when profiles are given.
 * Errors: LRBMS_E_ARG for inconsistent sizes, LRBMS_E_OOM, LRBMS_E_HIP.       */
int lrbms_model_create(const lrbms_problem* prob, const int32_t* basis_sizes,
                       const double* basis, int32_t n_profiles, const double* profiles,
                       lrbms_model** out);

/* Create a model whose local bases come from global snapshots (host,
 * [n_snap][r*ncell]): in every box, 1_E first when unit_functions is set, then
 * the restrictions of the snapshots in order, Gram-Schmidt in L2(E) (two
 * passes, rejection of remaining norms <= 1e-8 of the original), at most
 * ne_cap functions (Alg. 2 step 2e).  Profiles as in lrbms_model_create.     */
int lrbms_model_create_from_snapshots(const lrbms_problem* prob, int32_t n_snap,
                                      const double* snapshots, int32_t ne_cap,
                                      int32_t unit_functions, int32_t n_profiles,
                                      const double* profiles, lrbms_model** out);

/* Offline stage on the device (Alg. 2 steps 1-2 without the error-driven
 * selection): initial pressure by a fine SWIP solve (preconditioned CG),
 * velocity (Def. velocityDG), time-of-flight (eq. timeOfFlight, host
 * flow-ordered sweep), M profiles (Alg. 2 step 1c), fine snapshots at the
 * training mobilities, local Gram-Schmidt with 1_E first, cap N_E.
 * Untimed setup; its result is exported with lrbms_model_export_basis.        */
int lrbms_build_offline_bases(const lrbms_problem* prob, const lrbms_offline_opts* opts,
                              lrbms_model** out);

int lrbms_model_get_info(const lrbms_model* m, lrbms_model_info* info);

/* Copy the bases (host): sizes [n_sub], basis as in lrbms_model_create.       */
int lrbms_model_export_basis(const lrbms_model* m, int32_t* sizes, double* basis);

/* a) Mobility of d_sat (device, [r*ncell]) and the reduced system A_N, f_N
 *    (kept inside the model in block storage).  mode: LRBMS_DIRECT / _FIT / AFFINE. */
int lrbms_online_assemble(lrbms_model* m, const double* d_sat, int32_t mode, void* stream);

/* a) Factor A_N (multifrontal block Cholesky, nested-dissection order over the
 *    coarse boxes) and solve; d_pN (device, [N]) receives p_N.
 *    LRBMS_E_STATE if no assembly preceded.                                    */
int lrbms_online_solve(lrbms_model* m, double* d_pN, void* stream);

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
 * per-level work lists that the numeric kernels execute, flattened into
 * int64 records (layout documented in the Python binding).  With buf == NULL
 * or cap too small only *needed is set.  leaf_max: largest region (in boxes)
 * that becomes a leaf front.                                                   */
int lrbms_solver_plan_export(const lrbms_problem* prob, const int32_t* basis_sizes,
                             int32_t leaf_max, int64_t* buf, int64_t cap, int64_t* needed);

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

/* Synchronize and return the device status word (0 or a negative LRBMS_E_*). */
int lrbms_model_status(lrbms_model* m);

const char* lrbms_last_error(void);
void lrbms_model_destroy(lrbms_model* m);

#ifdef __cplusplus
}
#endif
#endif /* LRBMS_H */
