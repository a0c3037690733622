// Internal declarations of the LRBMS gfx950 library: device-side problem
// description, model layout and the launchers shared by the source files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lrbms.h"

namespace lrbms {

constexpr double kSqrt3 = 1.7320508075688772;
constexpr int kMaxProfiles = 64;

// Geometry, physics constants and problem arrays, passed by value to kernels.
struct Geom {
  int dim, r, n[3], ncell;
  int nfa[3], foff[3], nface;
  double h[3], vol, isv, area[3], hf[3], he;
  double visc_w, visc_o, cw, co;
  double ivw, ivo;   // 1 / visc_w, 1 / visc_o
  int relperm;
  double pen;        // penalty_c / max(visc_w, visc_o)
  int weights;
  double sat_pen;    // sat_penalty_scale
  int limiter;
  double dt;
  // dt max |f_w'| over [0, 1]: the transport step's CFL number of a cell is
  // cfl_coef times its outflow over phi |e|
  double cfl_coef;
  const double *perm, *poro, *q1, *q2, *bc_val, *bc_sval;
  const int8_t *bc_type, *bc_sat;
  // device status words: [0] the first error (atomicMin of LRBMS_E_* codes),
  // [1] a warning (LRBMS_W_CFL)
  int* status;
};

// CFL number above which a transport step raises LRBMS_W_CFL.
constexpr double kCflWarn = 0.5;

// One coarse box E.
struct Sub {
  int lo[3], hi[3];
  int nE, NE;        // cells, local basis size
  long long phi_off; // offset of Phi^E in the basis array
  int pn_off;        // offset of the box block in p_N
  long long blk_off; // offset of the diagonal block in block storage
};

// One coarse interface between box lo (low side along axis) and box hi.
struct Iface {
  int axis, lo, hi, nf;
  long long blk_off; // offset of A[lo][hi] (N_lo x N_hi, row-major)
  long long tr_off;  // offset of its face traces: lo side (N_lo, r, nf), then hi side (N_hi, r, nf)
};

// ---- device helpers ---------------------------------------------------------

// Workgroup b of a launch of n goes to XCD b mod 8 (the dispatcher hands
// them to the eight XCDs in turn, each XCD with an L2 of its own).  The work
// item a workgroup takes is renumbered so that every XCD works through one
// contiguous range of items: neighbouring items, which read the same input
// lines, then meet in the same L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_item(int b, int n) {
  const int per = n >> 3, rem = n & 7, x = b & 7, i = b >> 3;
  return x * per + min(x, rem) + i;
}
__device__ __forceinline__ double clip01(double s) { return fmin(fmax(s, 0.0), 1.0); }

// General Corey power, kept out of line: inlined at every mobility evaluation
// it would multiply the code of the kernels many times over (instruction
// cache misses) for a path that the quadratic exponents never take.
__device__ __noinline__ double corey_power(double s, double e) { return pow(s, e); }

__device__ __forceinline__ void mobilities(const Geom& g, double s, double& lw, double& lo) {
  const double sc = clip01(s);
  double krw, kro;
  if (g.relperm == 0) {
    krw = sc;
    kro = 1.0 - sc;
  } else {
    krw = (g.cw == 2.0) ? sc * sc : corey_power(sc, g.cw);
    const double so = 1.0 - sc;
    kro = (g.co == 2.0) ? so * so : corey_power(so, g.co);
  }
  lw = krw * g.ivw;
  lo = kro * g.ivo;
}

__device__ __forceinline__ double total_mobility(const Geom& g, double s) {
  double lw, lo;
  mobilities(g, s, lw, lo);
  return lw + lo;
}

// 1/d for a positive normal d: the hardware estimate y0 (relative error
// e = 1 - d y0 below 1e-7) refined to y0 (1 + e + e^2), whose error e^3 is
// below the rounding of a double.
__device__ __forceinline__ double rcp_refined(double d) {
  const double y0 = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, y0, 1.0);
  return fma(fma(e, e, e), y0, y0);
}

// Fractional flow f_w = lambda_w / (lambda_w + lambda_o); the total mobility
// is positive on [0, 1] (k_rw + k_ro > 0 for every law here).
__device__ __forceinline__ double frac_flow(const Geom& g, double s) {
  double lw, lo;
  mobilities(g, s, lw, lo);
  return lw * rcp_refined(lw + lo);
}

__device__ __forceinline__ void cell_coords(const Geom& g, int c, int x[3]) {
  x[0] = c % g.n[0];
  x[1] = (c / g.n[0]) % g.n[1];
  x[2] = c / (g.n[0] * g.n[1]);
}

__device__ __forceinline__ int cell_index(const Geom& g, const int x[3]) {
  return x[0] + g.n[0] * (x[1] + g.n[1] * x[2]);
}

// Global face number of the face along axis a at face coordinates x
// (x[a] in [0, n[a]]).
__device__ __forceinline__ int face_index(const Geom& g, int a, const int x[3]) {
  int e0 = g.n[0], e1 = g.n[1];
  if (a == 0) e0 += 1;
  if (a == 1) e1 += 1;
  return g.foff[a] + x[0] + e0 * (x[1] + e1 * x[2]);
}

// Number of mobility moment slots per cell: int_e gamma, then for every face
// side (axis a, dir 0 = low face, 1 = high face): int_f gamma and
// int_f gamma xi_t for the d-1 tangential axes t (in increasing order).
__host__ __device__ __forceinline__ int n_moments(int dim) { return 1 + 2 * dim * dim; }
__host__ __device__ __forceinline__ int mom_slot(int dim, int a, int dir) {
  return 1 + (2 * a + dir) * dim;
}

// ---- host helpers -------------------------------------------------------------
void set_error(const std::string& msg);
bool hip_ok(hipError_t e, const char* what);

// Launchers (defined in the .hip files).
enum GammaSource { GAMMA_SAT = 0, GAMMA_FIELD = 1, GAMMA_COMBO = 2 };
enum AsmParts { PART_GAMMA = 1, PART_PEN = 2, PART_RHS_CONST = 4, PART_RHS_GAMMA = 8 };

hipError_t launch_moments(const Geom& g, const double* src, int kind, const double* theta,
                          int nprof, long long prof_stride, double* mom, hipStream_t st);
// Work split of the box assembly: (box, first cell) chunks and partial blocks.
// variant 0: four waves, items of several columns per thread; 1: six waves,
// one (cell, column) item per thread (the autotuner picks per model).
struct AsmLayout {
  int* chunks = nullptr;       // [n_chunks][2] (box, first cell)
  int* first_chunk = nullptr;  // [n_sub + 1] first chunk of every box
  double* partial = nullptr;   // per-chunk partial blocks
  int n_chunks = 0;
  int variant = 0;
};
hipError_t assemble_prepare(const Geom& g, const std::vector<Sub>& subs, int max_ne,
                            int variant, AsmLayout& L, long long& bytes);
void assemble_free(AsmLayout& L);
hipError_t launch_assemble(const AsmLayout& L, const Geom& g, const Sub* d_subs, int n_sub,
                           int max_ne, const Iface* d_ifaces, int n_iface, const double* phi,
                           const double* tr, const double* mom, int parts, double* blocks,
                           double* fN, hipStream_t st);
// Face traces of the local bases per coarse interface (Iface::tr_off layout).
hipError_t launch_face_traces(const Geom& g, const Sub* d_subs, const Iface* d_ifaces, int n_iface,
                              const double* phi, double* tr, hipStream_t st);
hipError_t launch_affine_sum(const double* base, const double* terms, long long n,
                             const double* theta, int nq, double* out, hipStream_t st);
hipError_t launch_lsq(const Geom& g, const double* sat, const double* prof, int nprof,
                      const double* gchol, double* partial, int nblocks, double* theta,
                      hipStream_t st);
hipError_t launch_reconstruct(const Geom& g, const Sub* d_subs, int n_sub, const int* d_tiles,
                              int n_tiles, const double* phi, const double* pN, double* ph,
                              hipStream_t st);
hipError_t launch_flux(const Geom& g, const double* ph, const double* sat, double* flux,
                       hipStream_t st);
hipError_t launch_transport(const Geom& g, const double* sat, const double* flux,
                            double* sat_bar, hipStream_t st);
hipError_t launch_limiter(const Geom& g, const double* sat_bar, const double* flux,
                          double* sat_out, uint8_t* flags, hipStream_t st);
// Offline solvers (synchronous, default stream).  FineSolver: the fine SWIP
// pressure by multigrid-preconditioned CG, its work arrays and coarse
// hierarchy kept over solves of one problem (mom: moment scratch of the grid,
// d_status: device status word; warm: start from the contents of d_p).  tof_solve: the time of flight by
// block-Jacobi sweeps.  Return an LRBMS_* code.
struct FineSolver;
FineSolver* fine_solver_create(const Geom& g);
void fine_solver_destroy(FineSolver* S);
int fine_solver_solve(FineSolver* S, double* mom, const double* field, int kind, double rtol,
                      int maxit, bool warm, double* d_p, int* d_status, int* iters,
                      double* relres);
// Energy norm |a - b|^2 (b may be NULL) under b_h(., .; field), the field
// given once by fine_energy_setup (the greedy error measure).
int fine_energy_setup(FineSolver* S, double* mom, const double* field);
int fine_energy_diff(FineSolver* S, const double* a, const double* b, double* out);
int fine_energy_diff_batch(FineSolver* S, const double* a, long long as, const double* b,
                           long long bs, int n, double* out);
int tof_solve(const Geom& g, const double* d_flux, double tol, int maxit, double* d_tau,
              int* d_status, int* sweeps);
// The time of flight on caller-given work memory (no allocation):
// tof_scratch_doubles(g) doubles carved by tof_carve.
struct TofBufs { double *Minv, *C, *b, *other, *pc, *ps, *red; };
size_t tof_scratch_doubles(const Geom& g);
void tof_carve(const Geom& g, double* base, TofBufs& B);
int tof_solve_bufs(const Geom& g, const double* d_flux, double tol, int maxit, double* d_tau,
                   int* d_status, int* sweeps, const TofBufs& B);
// Padded column count of the assembly tiles (N_E + 1 rounded up to 16) and
// the number of workgroups of the least-squares projection.
int assemble_cols(int max_ne);
// Local bases of the device snapshots d_snaps ([nsnap][r*ncell]) in every
// box of subs: Gram-Schmidt (LRBMS_BASIS_GS, Alg. 2 step 2e) or the method
// of snapshots (LRBMS_BASIS_PCA with pca_eps, Alg. 2 step 3; at most 64
// snapshots).  sizes receives N_E per box, *d_basis a new device array of
// len doubles in the model's basis layout (the caller frees it).
// Synchronous.
int local_bases_device(const Geom& g, const std::vector<Sub>& subs, const double* d_snaps,
                       int nsnap, int cap, bool unit, int method, double pca_eps,
                       std::vector<int>& sizes, double** d_basis, long long& len);
// Local bases grown one function at a time on the device (the greedy
// extension of Alg. 2 step 2): room for cap functions per box.
struct DeviceBases;
void device_bases_free(DeviceBases& B);
struct DeviceBases {
  int cap = 0, n = 0;
  std::vector<int> sizes;              // functions per box (host copy)
  std::vector<long long> slot_off;     // first slot of each box
  Sub* d_subs = nullptr;
  long long* d_slot_off = nullptr;
  int* d_sizes = nullptr;
  double* d_slots = nullptr;
  DeviceBases() = default;
  DeviceBases(const DeviceBases&) = delete;
  DeviceBases& operator=(const DeviceBases&) = delete;
  ~DeviceBases() { device_bases_free(*this); }
};
int device_bases_init(const Geom& g, const std::vector<Sub>& subs, int cap, DeviceBases& B);
// Gram-Schmidt of the restrictions of d_snap ([r*ncell]) into every box's
// basis; grew: some box kept it.  Synchronous.
int device_bases_extend(const Geom& g, DeviceBases& B, const double* d_snap, bool& grew);
// The bases in the model layout: a new device array of len doubles.
int device_bases_compact(const Geom& g, const std::vector<Sub>& subs, const DeviceBases& B,
                         double** d_basis, long long& len);
int lsq_blocks(int ncell);

}  // namespace lrbms
