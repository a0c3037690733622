// Offline stage on gfx950 (Alg. 2 without the greedy selection):
//   * fine pressure solves of Def. pressureDG by conjugate gradients with
//     block-Jacobi preconditioning, the operator applied from per-cell r x r
//     stencil blocks formed once per mobility (the same discrete operator as
//     the online assembly, swip.h); scalars stay on the device and every
//     reduction runs in a fixed order;
//   * the DG time of flight of eq. timeOfFlight for given face fluxes by
//     block-Jacobi sweeps: each cell solves its r x r system with the upwind
//     traces of the previous sweep; on a flow without cycles the sweeps are
//     exact after as many sweeps as the longest upwind path has cells (the
//     flow-ordered block-triangular structure of the system, Sec. 3.6).
#include <memory>

#include "common.h"
#include "ktimer.h"
#include "swip.h"

namespace lrbms {

constexpr int kBlk = 256;

// Sum / maximum over the workgroup in a fixed order (every thread gets the
// result): butterfly within each wave, then the four wave results in order.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Neighbour of cell x across face f = 2a + dir, or -1 outside the grid.
__device__ __forceinline__ int face_neighbour(const Geom& g, const int (&x)[3], int f) {
  const int a = f >> 1, dir = f & 1;
  int y[3] = {x[0], x[1], x[2]};
  y[a] += dir ? 1 : -1;
  if (y[a] < 0 || y[a] >= g.n[a]) return -1;
  return cell_index(g, y);
}

// ---- fine SWIP operator ----------------------------------------------------
// K: per cell (1 + 2d) blocks of r x r (self, then one per face), entry
// ((f * r + k) * r + kp) of cell c at index entry * ncell + c.
template <int D>
__global__ __launch_bounds__(kBlk) void k_fine_stencil(Geom g, const double* __restrict__ mom,
                                                       double* __restrict__ K) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  const int item = blockIdx.x * kBlk + threadIdx.x;
  if (item >= nc * R) return;
  const int c = item % nc, kp = item / nc;
  int x[3];
  cell_coords(g, c, x);
  Sub S{};
  for (int a = 0; a < 3; ++a) {
    S.lo[a] = 0;
    S.hi[a] = g.n[a];
  }
  double self[R], nbr[2 * D][R];
  cell_stencil<D>(g, S, c, x, mom, PART_GAMMA | PART_PEN, kp, self, nbr);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    K[(size_t)(k * R + kp) * nc + c] = self[k];
#pragma unroll
    for (int f = 0; f < 2 * D; ++f) K[(size_t)(((1 + f) * R + k) * R + kp) * nc + c] = nbr[f][k];
  }
}

template <int D>
__global__ __launch_bounds__(kBlk) void k_fine_rhs(Geom g, const double* __restrict__ mom,
                                                   double* __restrict__ l) {
  constexpr int R = D + 1;
  const int c = blockIdx.x * kBlk + threadIdx.x;
  if (c >= g.ncell) return;
  int x[3];
  cell_coords(g, c, x);
  double Y[R];
#pragma unroll
  for (int k = 0; k < R; ++k) Y[k] = 0.0;
  cell_rhs<D>(g, c, x, mom, PART_RHS_CONST | PART_RHS_GAMMA, Y);
#pragma unroll
  for (int k = 0; k < R; ++k) l[(size_t)k * g.ncell + c] = Y[k];
}

// Inverse of an R x R matrix by Gauss-Jordan with partial pivoting; false if
// a pivot vanishes (the result is then the identity).
template <int R>
__device__ __forceinline__ bool small_inverse(double (&a)[R][R], double (&inv)[R][R]) {
  double w[R][2 * R];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      w[i][j] = a[i][j];
      w[i][R + j] = (i == j) ? 1.0 : 0.0;
    }
  bool ok = true;
#pragma unroll
  for (int col = 0; col < R; ++col) {
    // partial pivoting by swapping rows (static indices, selects only)
#pragma unroll
    for (int i = col + 1; i < R; ++i) {
      const bool sw = fabs(w[i][col]) > fabs(w[col][col]);
#pragma unroll
      for (int j = 0; j < 2 * R; ++j) {
        const double t = w[col][j];
        w[col][j] = sw ? w[i][j] : t;
        w[i][j] = sw ? t : w[i][j];
      }
    }
    double piv = w[col][col];
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) {
      ok = false;
      piv = 1.0;
    }
    const double ip = 1.0 / piv;
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) w[col][j] *= ip;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (i == col) continue;
      const double f = w[i][col];
#pragma unroll
      for (int j = 0; j < 2 * R; ++j) w[i][j] -= f * w[col][j];
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) inv[i][j] = ok ? w[i][R + j] : (i == j ? 1.0 : 0.0);
  return ok;
}

template <int D>
__global__ __launch_bounds__(kBlk) void k_fine_jacobi(Geom g, const double* __restrict__ K,
                                                      double* __restrict__ Dinv, int* status) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  const int c = blockIdx.x * kBlk + threadIdx.x;
  if (c >= nc) return;
  double a[R][R], inv[R][R];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) a[i][j] = K[(size_t)(i * R + j) * nc + c];
  if (!small_inverse<R>(a, inv)) atomicMin(status, (int)LRBMS_E_NOT_SPD);
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) Dinv[(size_t)(i * R + j) * nc + c] = inv[i][j];
}

// ---- multigrid-preconditioned conjugate gradients ----------------------------
// Preconditioner: one symmetric V-cycle.  Level 0 is the P1 DG space with
// damped cell-block Jacobi smoothing.  Level 1 is its subspace of cell-wise
// constants (coefficient 0 of every cell); the Galerkin operator there is the
// (0,0) entry of the stencil blocks, which only the penalty term produces
// (piecewise constants have no gradient), so the whole coarse hierarchy is
// independent of the mobility and is built once per problem.  Coarser levels
// aggregate 2^d cells (piecewise-constant prolongation, Galerkin operators that
// stay (2d+1)-point stencils); the coarsest (<= kMgCoarse cells) is solved with
// its dense inverse.  Pre- and post-smoothing are the same damped Jacobi
// step, so the V-cycle is symmetric positive definite when the damping keeps
// the smoother convergent.
//
// CG keeps its scalars on the device: every workgroup sums the
// per-workgroup partials of the previous launch itself, in the same fixed
// order, so all workgroups see identical alpha and beta.  Ap is carried by
// the recursion A p_new = A z + beta A p_old.  The grid is capped
// (grid-stride loops) to bound the partial sums.
constexpr int kCgMaxBlocks = 1024;
constexpr int kMgCoarse = 512;
// Damped Jacobi on the P0 levels (diagonally dominant, so the eigenvalues of
// D^-1 A lie in [0, 2]); level-0 damping relative to the estimated largest
// eigenvalue of D^-1 A; over-relaxed coarse corrections, which compensate the
// weak piecewise-constant prolongation (values chosen by convergence tests on
// the configured problems; each keeps the V-cycle symmetric positive definite).
constexpr double kMgOmega = 0.8;
constexpr double kMgOmega0 = 1.5;
constexpr double kMgAlpha0 = 1.3;   // level 1 -> level 0
constexpr double kMgAlpha = 1.7;    // level l+1 -> level l

__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlk) s += p[i];
  return block_sum(s, red);
}

// Apply the cell's r x r blocks (rows k0 .. k1-1) to v.
template <int D, int K0, int K1>
__device__ __forceinline__ void stencil_rows(const Geom& g, const double* __restrict__ K,
                                             const double (&u)[1 + 2 * D][D + 1], int c,
                                             double (&y)[D + 1]) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    double s = 0.0;
#pragma unroll
    for (int f = 0; f < 1 + 2 * D; ++f)
#pragma unroll
      for (int kp = 0; kp < R; ++kp) s = fma(K[(size_t)((f * R + k) * R + kp) * nc + c], u[f][kp], s);
    y[k] = s;
  }
}

// Coefficients of v on the cell and its face neighbours (zero outside).
template <int D>
__device__ __forceinline__ void gather(const Geom& g, const double* __restrict__ v, int c,
                                       const int (&xc)[3], double (&u)[1 + 2 * D][D + 1]) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
#pragma unroll
  for (int k = 0; k < R; ++k) u[0][k] = v[(size_t)k * nc + c];
#pragma unroll
  for (int f = 0; f < 2 * D; ++f) {
    const int n = face_neighbour(g, xc, f);
#pragma unroll
    for (int k = 0; k < R; ++k) u[1 + f][k] = (n >= 0) ? v[(size_t)k * nc + n] : 0.0;
  }
}

// w = omega * Dinv_c r_c  (+ e on coefficient 0)
template <int D>
__device__ __forceinline__ void jacobi_cell(const Geom& g, const double* __restrict__ Dinv,
                                            const double* __restrict__ r, double omega, int c,
                                            double e0, double (&w)[D + 1]) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  double rv[R];
#pragma unroll
  for (int k = 0; k < R; ++k) rv[k] = r[(size_t)k * nc + c];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) t = fma(Dinv[(size_t)(i * R + j) * nc + c], rv[j], t);
    w[i] = omega * t;
  }
  w[0] += e0;
}

// Level 1 stencil: the (0,0) entries of the self and face blocks.
template <int D>
__global__ __launch_bounds__(kBlk) void k_mg_extract(Geom g, const double* __restrict__ K,
                                                     double* __restrict__ diag,
                                                     double* __restrict__ off) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += gridDim.x * kBlk) {
    diag[c] = K[c];
#pragma unroll
    for (int f = 0; f < 2 * D; ++f) off[(size_t)f * nc + c] = K[(size_t)((1 + f) * R * R) * nc + c];
  }
}

// Level 0 down: z0 = omega0 D^-1 r, level-1 right-hand side = coefficient 0 of
// r - A z0.
template <int D>
__global__ __launch_bounds__(kBlk) void k_mg0_down(Geom g, const double* __restrict__ K,
                                                   const double* __restrict__ Dinv,
                                                   const double* __restrict__ r, double omega0,
                                                   double* __restrict__ b1) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += gridDim.x * kBlk) {
    int xc[3];
    cell_coords(g, c, xc);
    double u[1 + 2 * D][R];
    jacobi_cell<D>(g, Dinv, r, omega0, c, 0.0, u[0]);
#pragma unroll
    for (int f = 0; f < 2 * D; ++f) {
      const int n = face_neighbour(g, xc, f);
      if (n >= 0) {
        jacobi_cell<D>(g, Dinv, r, omega0, n, 0.0, u[1 + f]);
      } else {
#pragma unroll
        for (int k = 0; k < R; ++k) u[1 + f][k] = 0.0;
      }
    }
    double y[R];
    stencil_rows<D, 0, 1>(g, K, u, c, y);
    b1[c] = r[c] - y[0];
  }
}

// Level 0 up: z = z0 + alpha0 e1 (on coefficient 0), then z += omega0 D^-1 (r - A z);
// partials of r . z.
template <int D>
__global__ __launch_bounds__(kBlk) void k_mg0_up(Geom g, const double* __restrict__ K,
                                                 const double* __restrict__ Dinv,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ e1, double omega0,
                                                 double* __restrict__ z,
                                                 double* __restrict__ part_rz) {
  constexpr int R = D + 1;
  __shared__ double red[4];
  const int nc = g.ncell;
  double rz = 0.0;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += gridDim.x * kBlk) {
    int xc[3];
    cell_coords(g, c, xc);
    double u[1 + 2 * D][R];
    jacobi_cell<D>(g, Dinv, r, omega0, c, kMgAlpha0 * e1[c], u[0]);
#pragma unroll
    for (int f = 0; f < 2 * D; ++f) {
      const int n = face_neighbour(g, xc, f);
      if (n >= 0) {
        jacobi_cell<D>(g, Dinv, r, omega0, n, kMgAlpha0 * e1[n], u[1 + f]);
      } else {
#pragma unroll
        for (int k = 0; k < R; ++k) u[1 + f][k] = 0.0;
      }
    }
    double y[R], res[R];
    stencil_rows<D, 0, R>(g, K, u, c, y);
#pragma unroll
    for (int k = 0; k < R; ++k) res[k] = r[(size_t)k * nc + c] - y[k];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) t = fma(Dinv[(size_t)(i * R + j) * nc + c], res[j], t);
      const double zi = fma(omega0, t, u[0][i]);
      z[(size_t)i * nc + c] = zi;
      rz = fma(r[(size_t)i * nc + c], zi, rz);
    }
  }
  const double t = block_sum(rz, red);
  if (threadIdx.x == 0) part_rz[blockIdx.x] = t;
}

// One P0 level: cells m[0] x m[1] x m[2], x fastest.
struct MgGrid {
  int m[3], n;
};

__device__ __forceinline__ int mg_neighbour(const MgGrid& L, const int (&x)[3], int f) {
  const int a = f >> 1;
  int y[3] = {x[0], x[1], x[2]};
  y[a] += (f & 1) ? 1 : -1;
  if (y[a] < 0 || y[a] >= L.m[a]) return -1;
  return y[0] + L.m[0] * (y[1] + L.m[1] * y[2]);
}

__device__ __forceinline__ void mg_coords(const MgGrid& L, int c, int (&x)[3]) {
  x[0] = c % L.m[0];
  x[1] = (c / L.m[0]) % L.m[1];
  x[2] = c / (L.m[0] * L.m[1]);
}

__device__ __forceinline__ int mg_parent(const MgGrid& C, const int (&x)[3]) {
  return (x[0] >> 1) + C.m[0] * ((x[1] >> 1) + C.m[1] * (x[2] >> 1));
}

// Level l down for coarse cell q: e = omega b / d on every cell of its
// aggregate, coarse right-hand side = sum over the aggregate of b - A e.
// (b may live in LDS or in global memory.)
template <int D>
__device__ __forceinline__ double mg_down_value(const MgGrid& L, const MgGrid& C,
                                                const double* __restrict__ diag,
                                                const double* __restrict__ off,
                                                const double* b, int q) {
  int X[3];
  mg_coords(C, q, X);
  double sum = 0.0;
#pragma unroll
  for (int ch = 0; ch < (1 << D); ++ch) {
    const int x[3] = {2 * X[0] + (ch & 1), 2 * X[1] + ((ch >> 1) & 1),
                      D == 3 ? 2 * X[2] + ((ch >> 2) & 1) : 0};
    if (x[0] >= L.m[0] || x[1] >= L.m[1] || x[2] >= L.m[2]) continue;
    const int c = x[0] + L.m[0] * (x[1] + L.m[1] * x[2]);
    const double bcv = b[c];
    double res = bcv - kMgOmega * bcv;
#pragma unroll
    for (int f = 0; f < 2 * D; ++f) {
      const int n = mg_neighbour(L, x, f);
      if (n >= 0) res -= off[(size_t)f * L.n + c] * (kMgOmega * b[n] / diag[n]);
    }
    sum += res;
  }
  return sum;
}

// Level l up for cell c: e = omega b / d + alpha P e_coarse, then
// e += omega (b - A e) / d.
template <int D>
__device__ __forceinline__ double mg_up_value(const MgGrid& L, const MgGrid& C,
                                              const double* __restrict__ diag,
                                              const double* __restrict__ off, const double* b,
                                              const double* ec, int c) {
  int x[3];
  mg_coords(L, c, x);
  const double dc = diag[c];
  const double ev = kMgOmega * b[c] / dc + kMgAlpha * ec[mg_parent(C, x)];
  double res = b[c] - dc * ev;
#pragma unroll
  for (int f = 0; f < 2 * D; ++f) {
    const int n = mg_neighbour(L, x, f);
    if (n < 0) continue;
    int y[3];
    mg_coords(L, n, y);
    res -= off[(size_t)f * L.n + c] * (kMgOmega * b[n] / diag[n] + kMgAlpha * ec[mg_parent(C, y)]);
  }
  return ev + kMgOmega * res / dc;
}

template <int D>
__global__ __launch_bounds__(kBlk) void k_mgl_down(MgGrid L, MgGrid C,
                                                   const double* __restrict__ diag,
                                                   const double* __restrict__ off,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ bc) {
  for (int q = blockIdx.x * kBlk + threadIdx.x; q < C.n; q += gridDim.x * kBlk)
    bc[q] = mg_down_value<D>(L, C, diag, off, b, q);
}

template <int D>
__global__ __launch_bounds__(kBlk) void k_mgl_up(MgGrid L, MgGrid C,
                                                 const double* __restrict__ diag,
                                                 const double* __restrict__ off,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ ec,
                                                 double* __restrict__ e) {
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < L.n; c += gridDim.x * kBlk)
    e[c] = mg_up_value<D>(L, C, diag, off, b, ec, c);
}

// The small levels of the V-cycle in one workgroup: from level t (at most
// kTailCells cells) down to the coarsest, the dense coarse solve, and back up
// to level t, with every level's b and e in LDS (barriers between the levels
// instead of launches).
constexpr int kTailCells = 4096;
constexpr int kTailLevels = 8;
constexpr int kTailThreads = 1024;
struct TailDesc {
  int nt;                               // levels t .. t+nt-1 (the last is the coarsest)
  MgGrid grid[kTailLevels];
  const double* diag[kTailLevels];
  const double* off[kTailLevels];
  int lds[kTailLevels];                 // offset of the level's b (its e follows)
};

template <int D>
__global__ __launch_bounds__(kTailThreads) void k_mg_tail(TailDesc T,
                                                          const double* __restrict__ inv,
                                                          const double* __restrict__ bt,
                                                          double* __restrict__ et) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x;
  const int n0 = T.grid[0].n;
  for (int c = tid; c < n0; c += kTailThreads) sm[T.lds[0] + c] = bt[c];
  __syncthreads();
  for (int k = 0; k + 1 < T.nt; ++k) {
    const double* b = sm + T.lds[k];
    double* bc = sm + T.lds[k + 1];
    for (int q = tid; q < T.grid[k + 1].n; q += kTailThreads)
      bc[q] = mg_down_value<D>(T.grid[k], T.grid[k + 1], T.diag[k], T.off[k], b, q);
    __syncthreads();
  }
  {
    // coarsest: e = A^-1 b.  Thread (row i, column quarter q) sums a quarter
    // of row i (inv holds A^-1 transposed, so the reads are coalesced over i);
    // the quarters meet in LDS in a fixed order.
    const int k = T.nt - 1, n = T.grid[k].n;
    const double* b = sm + T.lds[k];
    double* e = sm + T.lds[k] + n;
    double* part = sm + T.lds[k] + 2 * n;   // 4 n doubles past the last level
    const int nq = (n + 3) / 4;
    for (int w = tid; w < 4 * n; w += kTailThreads) {
      const int i = w % n, q = w / n;
      const int j0 = q * nq, j1 = min(n, j0 + nq);
      double s = 0.0;
      for (int j = j0; j < j1; ++j) s = fma(inv[(size_t)j * n + i], b[j], s);
      part[q * n + i] = s;
    }
    __syncthreads();
    for (int i = tid; i < n; i += kTailThreads)
      e[i] = (part[i] + part[n + i]) + (part[2 * n + i] + part[3 * n + i]);
    __syncthreads();
  }
  for (int k = T.nt - 2; k >= 0; --k) {
    const int n = T.grid[k].n;
    const double* b = sm + T.lds[k];
    const double* ec = sm + T.lds[k + 1] + T.grid[k + 1].n;
    double* e = sm + T.lds[k] + n;
    for (int c = tid; c < n; c += kTailThreads)
      e[c] = mg_up_value<D>(T.grid[k], T.grid[k + 1], T.diag[k], T.off[k], b, ec, c);
    __syncthreads();
  }
  for (int c = tid; c < n0; c += kTailThreads) et[c] = sm[T.lds[0] + n0 + c];
}

// Power iteration for the largest eigenvalue of D^-1 A: w = D^-1 A (v * scale);
// partials of |w|^2.
template <int D>
__global__ __launch_bounds__(kBlk) void k_power(Geom g, const double* __restrict__ K,
                                                const double* __restrict__ Dinv,
                                                const double* __restrict__ v, double scale,
                                                double* __restrict__ w,
                                                double* __restrict__ part) {
  constexpr int R = D + 1;
  __shared__ double red[4];
  const int nc = g.ncell;
  double acc = 0.0;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += gridDim.x * kBlk) {
    int xc[3];
    cell_coords(g, c, xc);
    double u[1 + 2 * D][R];
    gather<D>(g, v, c, xc, u);
    double y[R];
    stencil_rows<D, 0, R>(g, K, u, c, y);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) t = fma(Dinv[(size_t)(i * R + j) * nc + c], y[j], t);
      t *= scale;
      w[(size_t)i * nc + c] = t;
      acc = fma(t, t, acc);
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlk) void k_power_start(long long n, double* __restrict__ v) {
  const long long i = blockIdx.x * (long long)kBlk + threadIdx.x;
  if (i >= n) return;
  // a fixed, non-special start vector: values in [0.5, 1.5)
  unsigned long long h = (unsigned long long)i * 0x9E3779B97F4A7C15ull;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  v[i] = 0.5 + (double)(h >> 11) * 0x1.0p-53;
}

// r = b - A x (WARM: x as given) or x = 0, r = b; partials of r . r and b . b.
template <int D, bool WARM>
__global__ __launch_bounds__(kBlk) void k_cg_init(Geom g, const double* __restrict__ K,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ part_rr,
                                                  double* __restrict__ part_bb) {
  constexpr int R = D + 1;
  __shared__ double red[4];
  const int nc = g.ncell;
  double rr = 0.0, bb = 0.0;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += gridDim.x * kBlk) {
    double ax[R];
    if (WARM) {
      int xc[3];
      cell_coords(g, c, xc);
      double u[1 + 2 * D][R];
      gather<D>(g, x, c, xc, u);
      stencil_rows<D, 0, R>(g, K, u, c, ax);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const double v = b[(size_t)k * nc + c];
      const double rv = WARM ? v - ax[k] : v;
      if (!WARM) x[(size_t)k * nc + c] = 0.0;
      r[(size_t)k * nc + c] = rv;
      rr = fma(rv, rv, rr);
      bb = fma(v, v, bb);
    }
  }
  const double t = block_sum(rr, red);
  const double t2 = block_sum(bb, red);
  if (threadIdx.x == 0) {
    part_rr[blockIdx.x] = t;
    part_bb[blockIdx.x] = t2;
  }
}

// beta = (r.z)_new / (r.z)_old (0 on the first iteration); p = z + beta p,
// Ap = A z + beta Ap; partials of p.Ap.
template <int D, bool FIRST>
__global__ __launch_bounds__(kBlk) void k_cg_direction(Geom g, const double* __restrict__ K,
                                                       const double* __restrict__ z,
                                                       double* __restrict__ p,
                                                       double* __restrict__ Ap,
                                                       const double* __restrict__ rz_new,
                                                       const double* __restrict__ rz_old,
                                                       double* __restrict__ part_pap) {
  constexpr int R = D + 1;
  __shared__ double red[4];
  const int nc = g.ncell, nb = gridDim.x;
  double beta = 0.0;
  if (!FIRST) {
    const double num = sum_partials(rz_new, nb, red);
    const double den = sum_partials(rz_old, nb, red);
    beta = den != 0.0 ? num / den : 0.0;
  }
  double dot = 0.0;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += nb * kBlk) {
    int xc[3];
    cell_coords(g, c, xc);
    double u[1 + 2 * D][R];
    gather<D>(g, z, c, xc, u);
    double w[R];
    stencil_rows<D, 0, R>(g, K, u, c, w);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const size_t i = (size_t)k * nc + c;
      const double pk = FIRST ? u[0][k] : fma(beta, p[i], u[0][k]);
      const double ak = FIRST ? w[k] : fma(beta, Ap[i], w[k]);
      p[i] = pk;
      Ap[i] = ak;
      dot = fma(pk, ak, dot);
    }
  }
  const double t = block_sum(dot, red);
  if (threadIdx.x == 0) part_pap[blockIdx.x] = t;
}

// alpha = (r.z) / (p.Ap); x += alpha p, r -= alpha Ap; partials of r.r.  A
// non-positive or non-finite curvature or r.z sets fail.
template <int D>
__global__ __launch_bounds__(kBlk) void k_cg_update(Geom g, double* __restrict__ x,
                                                    double* __restrict__ r,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ Ap,
                                                    const double* __restrict__ rz_cur,
                                                    const double* __restrict__ part_pap,
                                                    double* __restrict__ part_rr,
                                                    int* __restrict__ fail) {
  constexpr int R = D + 1;
  __shared__ double red[4];
  const int nc = g.ncell, nb = gridDim.x;
  const double rz = sum_partials(rz_cur, nb, red);
  const double pap = sum_partials(part_pap, nb, red);
  const bool ok = pap > 0.0 && isfinite(pap) && rz >= 0.0;
  const double al = ok ? rz / pap : 0.0;
  if (!ok && blockIdx.x == 0 && threadIdx.x == 0) *fail = 1;
  double rr = 0.0;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += nb * kBlk) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const size_t i = (size_t)k * nc + c;
      x[i] = fma(al, p[i], x[i]);
      const double rv = fma(-al, Ap[i], r[i]);
      r[i] = rv;
      rr = fma(rv, rv, rr);
    }
  }
  const double t = block_sum(rr, red);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = t;
}

// ---- energy norm of the greedy error measure ---------------------------------
// partials of e . (A e) for the operator held in K
template <int D>
__global__ __launch_bounds__(kBlk) void k_energy(Geom g, const double* __restrict__ K,
                                                 const double* __restrict__ e,
                                                 double* __restrict__ part) {
  constexpr int R = D + 1;
  __shared__ double red[4];
  const int nc = g.ncell;
  double acc = 0.0;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += gridDim.x * kBlk) {
    int xc[3];
    cell_coords(g, c, xc);
    double u[1 + 2 * D][R];
    gather<D>(g, e, c, xc, u);
    double y[R];
    stencil_rows<D, 0, R>(g, K, u, c, y);
#pragma unroll
    for (int k = 0; k < R; ++k) acc = fma(u[0][k], y[k], acc);
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlk) void k_diff(long long n, const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               double* __restrict__ out) {
  const long long i = blockIdx.x * (long long)kBlk + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

// ---- time of flight -----------------------------------------------------------
// Per cell: Minv (r x r, the inverse of the cell block: volume term with the
// RT0 velocity of the face fluxes and the own trace on outflow faces), C (one
// r x r block per face: the upwind neighbour's trace on inflow faces), b (the
// porosity term).
template <int D>
__global__ __launch_bounds__(kBlk) void k_tof_setup(Geom g, const double* __restrict__ F,
                                                    double* __restrict__ Minv,
                                                    double* __restrict__ C,
                                                    double* __restrict__ b, int* status) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  const int c = blockIdx.x * kBlk + threadIdx.x;
  if (c >= nc) return;
  int x[3];
  cell_coords(g, c, x);
  double M[R][R];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) M[i][j] = 0.0;
  const double iv = 1.0 / g.vol;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int xh[3] = {x[0], x[1], x[2]};
    xh[a] += 1;
    const double Flo = F[face_index(g, a, x)], Fhi = F[face_index(g, a, xh)];
    // -int_e tau u . grad psi with u_a = ub + dl xi_a (RT0), psi = phi_{a+1}
    const double ub = 0.5 * (Flo + Fhi) / g.area[a], dl = 0.5 * (Fhi - Flo) / g.area[a];
    M[a + 1][0] -= 2.0 * kSqrt3 / g.h[a] * ub;
    M[a + 1][a + 1] -= 2.0 / g.h[a] * dl;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const double sg = dir ? 1.0 : -1.0;
      const double fo = dir ? Fhi : -Flo;   // outward flux of this face
      const double wgt = fo * iv;           // (u.n) int_f phi phi = F_out / |e| * (trace table)
      double T[R][R];
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) T[i][j] = 0.0;
      const int f = 2 * a + dir;
      const int n = face_neighbour(g, x, f);
      if (fo >= 0.0) {
        // own trace: phi_0 = |e|^-1/2, phi_{a+1} = sqrt(3) sg |e|^-1/2, tangential mean zero
        T[0][0] = 1.0;
        T[0][a + 1] = T[a + 1][0] = kSqrt3 * sg;
        T[a + 1][a + 1] = 3.0;
#pragma unroll
        for (int t = 0; t < D; ++t)
          if (t != a) T[t + 1][t + 1] = 1.0;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int j = 0; j < R; ++j) M[i][j] += wgt * T[i][j];
      } else if (n >= 0) {
        // neighbour trace (its normal coordinate is -sg on this face)
        T[0][0] = 1.0;
        T[0][a + 1] = -kSqrt3 * sg;
        T[a + 1][0] = kSqrt3 * sg;
        T[a + 1][a + 1] = -3.0;
#pragma unroll
        for (int t = 0; t < D; ++t)
          if (t != a) T[t + 1][t + 1] = 1.0;
      }
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j)
          C[(size_t)((f * R + i) * R + j) * nc + c] = (fo < 0.0 && n >= 0) ? wgt * T[i][j] : 0.0;
    }
  }
  double inv[R][R];
  if (!small_inverse<R>(M, inv)) atomicMin(status, (int)LRBMS_E_NOT_SPD);
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) Minv[(size_t)(i * R + j) * nc + c] = inv[i][j];
  b[c] = g.poro[c] * sqrt(g.vol);
#pragma unroll
  for (int k = 1; k < R; ++k) b[(size_t)k * nc + c] = 0.0;
}

// One sweep: tau_new = Minv (b - sum_f C_f tau_old(neighbour)); block maxima
// of |tau_new - tau_old| and |tau_new|.
template <int D>
__global__ __launch_bounds__(kBlk) void k_tof_sweep(Geom g, const double* __restrict__ Minv,
                                                    const double* __restrict__ C,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ t_old,
                                                    double* __restrict__ t_new,
                                                    double* __restrict__ part_change,
                                                    double* __restrict__ part_size) {
  constexpr int R = D + 1;
  __shared__ double red[kBlk];
  const int nc = g.ncell;
  const int c = blockIdx.x * kBlk + threadIdx.x;
  double chg = 0.0, siz = 0.0;
  if (c < nc) {
    int x[3];
    cell_coords(g, c, x);
    double rhs[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rhs[k] = b[(size_t)k * nc + c];
#pragma unroll
    for (int f = 0; f < 2 * D; ++f) {
      const int n = face_neighbour(g, x, f);
      if (n < 0) continue;
      double tn[R];
#pragma unroll
      for (int k = 0; k < R; ++k) tn[k] = t_old[(size_t)k * nc + n];
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) rhs[i] = fma(-C[(size_t)((f * R + i) * R + j) * nc + c], tn[j], rhs[i]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) s = fma(Minv[(size_t)(i * R + j) * nc + c], rhs[j], s);
      const size_t idx = (size_t)i * nc + c;
      chg = fmax(chg, fabs(s - t_old[idx]));
      siz = fmax(siz, fabs(s));
      t_new[idx] = s;
    }
  }
  const double m1 = block_max(chg, red);
  const double m2 = block_max(siz, red);
  if (threadIdx.x == 0) {
    part_change[blockIdx.x] = m1;
    part_size[blockIdx.x] = m2;
  }
}

// ---- host drivers --------------------------------------------------------------
struct DevBuf {
  double* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  bool alloc(size_t n) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(double)) == hipSuccess;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

static int blocks_for(long long n) { return (int)((n + kBlk - 1) / kBlk); }

static double host_sum(const std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s += x;
  return s;
}

// Fine pressure solver of one problem: work arrays and the mobility-free
// coarse hierarchy, reused over solves with different mobilities.
struct FineSolver {
  Geom g{};
  int nb = 0, nbc = 0;
  DevBuf K, Dinv, l, r, z, pv, Ap, prz, prr, ppap, fl, mg, cinv;
  DevBuf Kbar, ework;                  // operator of the energy norm, difference vector
  bool have_bar = false;
  std::vector<MgGrid> grids;           // P0 levels 1 .. L
  std::vector<double*> diag, off, b, e;
  int tail_start = 0;                  // first level of the single-workgroup tail
  TailDesc tail{};
  size_t tail_lds = 0;
  bool have_mg = false;
};

// Dense inverse of the SPD matrix A (n x n, row-major, in place) by Cholesky.
static bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = v / d;
    }
  }
  std::vector<double> y(n), x(n);
  for (int col = 0; col < n; ++col) {
    for (int i = 0; i < n; ++i) {
      double v = (i == col) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * y[k];
      y[i] = v / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * x[k];
      x[i] = v / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) A[(size_t)i * n + col] = x[i];
  }
  return true;
}

// Coarse hierarchy from the level-1 stencil (the (0,0) entries of K).
template <int D>
static int build_hierarchy(FineSolver& S) {
  const Geom& g = S.g;
  S.grids.clear();
  MgGrid L1{{g.n[0], g.n[1], g.n[2]}, g.ncell};
  S.grids.push_back(L1);
  while (S.grids.back().n > kMgCoarse && S.grids.size() < 24) {
    MgGrid C = S.grids.back();
    for (int a = 0; a < D; ++a) C.m[a] = (C.m[a] + 1) / 2;
    C.n = C.m[0] * C.m[1] * C.m[2];
    S.grids.push_back(C);
  }
  const int nl = (int)S.grids.size();
  size_t total = 0;
  for (auto& G : S.grids) total += (size_t)(3 + 2 * D) * G.n;
  if (!S.mg.alloc(total)) return LRBMS_E_OOM;
  S.diag.assign(nl, nullptr);
  S.off.assign(nl, nullptr);
  S.b.assign(nl, nullptr);
  S.e.assign(nl, nullptr);
  size_t o = 0;
  for (int l = 0; l < nl; ++l) {
    const size_t n = S.grids[l].n;
    S.diag[l] = S.mg.p + o;
    S.off[l] = S.diag[l] + n;
    S.b[l] = S.off[l] + 2 * D * n;
    S.e[l] = S.b[l] + n;
    o += (size_t)(3 + 2 * D) * n;
  }
  hipLaunchKernelGGL(k_mg_extract<D>, dim3(std::min(blocks_for(g.ncell), 4096)), dim3(kBlk), 0, 0,
                     g, S.K.p, S.diag[0], S.off[0]);
  std::vector<double> hd(g.ncell), ho((size_t)2 * D * g.ncell);
  if (hipMemcpy(hd.data(), S.diag[0], hd.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(ho.data(), S.off[0], ho.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return LRBMS_E_HIP;
  for (int l = 0; l + 1 < nl; ++l) {
    const MgGrid& F = S.grids[l];
    const MgGrid& C = S.grids[l + 1];
    std::vector<double> cd(C.n, 0.0), co((size_t)2 * D * C.n, 0.0);
    for (int c = 0; c < F.n; ++c) {
      const int x[3] = {c % F.m[0], (c / F.m[0]) % F.m[1], c / (F.m[0] * F.m[1])};
      const int P = (x[0] >> 1) + C.m[0] * ((x[1] >> 1) + C.m[1] * (x[2] >> 1));
      cd[P] += hd[c];
      for (int f = 0; f < 2 * D; ++f) {
        const int a = f >> 1;
        int y[3] = {x[0], x[1], x[2]};
        y[a] += (f & 1) ? 1 : -1;
        if (y[a] < 0 || y[a] >= F.m[a]) continue;
        const int Q = (y[0] >> 1) + C.m[0] * ((y[1] >> 1) + C.m[1] * (y[2] >> 1));
        const double v = ho[(size_t)f * F.n + c];
        if (Q == P) cd[P] += v;
        else co[(size_t)f * C.n + P] += v;
      }
    }
    if (hipMemcpy(S.diag[l + 1], cd.data(), cd.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S.off[l + 1], co.data(), co.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return LRBMS_E_HIP;
    hd.swap(cd);
    ho.swap(co);
  }
  // dense inverse of the coarsest level
  const MgGrid& Cg = S.grids.back();
  const int n = Cg.n;
  std::vector<double> A((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    const int x[3] = {c % Cg.m[0], (c / Cg.m[0]) % Cg.m[1], c / (Cg.m[0] * Cg.m[1])};
    A[(size_t)c * n + c] = hd[c];
    for (int f = 0; f < 2 * D; ++f) {
      const int a = f >> 1;
      int y[3] = {x[0], x[1], x[2]};
      y[a] += (f & 1) ? 1 : -1;
      if (y[a] < 0 || y[a] >= Cg.m[a]) continue;
      A[(size_t)c * n + y[0] + Cg.m[0] * (y[1] + Cg.m[1] * y[2])] = ho[(size_t)f * n + c];
    }
  }
  if (!spd_inverse(A, n)) return LRBMS_E_NOT_SPD;
  // the tail: levels from the first with at most kTailCells cells
  int t = 0;
  while (S.grids[t].n > kTailCells) ++t;
  t = std::max(t, nl - kTailLevels);
  S.tail_start = t;
  S.tail = TailDesc{};
  S.tail.nt = nl - t;
  size_t lds = 0;
  for (int k = 0; k < S.tail.nt; ++k) {
    S.tail.grid[k] = S.grids[t + k];
    S.tail.diag[k] = S.diag[t + k];
    S.tail.off[k] = S.off[t + k];
    S.tail.lds[k] = (int)lds;
    lds += 2 * (size_t)S.grids[t + k].n;
  }
  lds += 4 * (size_t)S.grids[nl - 1].n;   // partial sums of the coarse solve
  S.tail_lds = lds * sizeof(double);
  if (S.tail_lds > 160 * 1024) return LRBMS_E_ARG;
  if (hipFuncSetAttribute((const void*)k_mg_tail<D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)S.tail_lds) != hipSuccess)
    return LRBMS_E_HIP;
  std::vector<double> At((size_t)n * n);   // transposed: At[j n + i] = (A^-1)_ij
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) At[(size_t)j * n + i] = A[(size_t)i * n + j];
  if (!S.cinv.alloc((size_t)n * n)) return LRBMS_E_OOM;
  if (hipMemcpy(S.cinv.p, At.data(), At.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return LRBMS_E_HIP;
  S.have_mg = true;
  return LRBMS_OK;
}

// z = B r (one V-cycle); partials of r . z.
template <int D>
static void vcycle(FineSolver& S, double omega0, const double* r, double* z, double* part_rz) {
  const Geom& g = S.g;
  hipLaunchKernelGGL(k_mg0_down<D>, dim3(std::min(blocks_for(g.ncell), 8192)), dim3(kBlk), 0, 0,
                     g, S.K.p, S.Dinv.p, r, omega0, S.b[0]);
  const int t = S.tail_start;
  for (int l = 0; l < t; ++l)
    hipLaunchKernelGGL(k_mgl_down<D>, dim3(std::min(blocks_for(S.grids[l + 1].n), 8192)),
                       dim3(kBlk), 0, 0, S.grids[l], S.grids[l + 1], S.diag[l], S.off[l], S.b[l],
                       S.b[l + 1]);
  hipLaunchKernelGGL(k_mg_tail<D>, dim3(1), dim3(kTailThreads), S.tail_lds, 0, S.tail, S.cinv.p,
                     S.b[t], S.e[t]);
  for (int l = t - 1; l >= 0; --l)
    hipLaunchKernelGGL(k_mgl_up<D>, dim3(std::min(blocks_for(S.grids[l].n), 8192)), dim3(kBlk), 0,
                       0, S.grids[l], S.grids[l + 1], S.diag[l], S.off[l], S.b[l], S.e[l + 1],
                       S.e[l]);
  hipLaunchKernelGGL(k_mg0_up<D>, dim3(S.nbc), dim3(kBlk), 0, 0, g, S.K.p, S.Dinv.p, r, S.e[0],
                     omega0, z, part_rz);
}

template <int D>
static int fine_solve_t(FineSolver& S, double* mom, const double* field, int kind, double rtol,
                        int maxit, bool warm, double* d_p, int* d_status, int* iters,
                        double* relres) {
  constexpr int R = D + 1;
  const Geom& g = S.g;
  const int nc = g.ncell, nb = S.nb, nbc = S.nbc;
  const size_t n = (size_t)R * nc;
  hipStream_t st = 0;
  int* d_fail = reinterpret_cast<int*>(S.fl.p);
  if (hipMemset(d_fail, 0, sizeof(int)) != hipSuccess) return LRBMS_E_HIP;
  if (launch_moments(g, field, kind, nullptr, 0, 0, mom, st) != hipSuccess) return LRBMS_E_HIP;
  hipLaunchKernelGGL(k_fine_stencil<D>, dim3(blocks_for((long long)nc * R)), dim3(kBlk), 0, st, g,
                     mom, S.K.p);
  hipLaunchKernelGGL(k_fine_rhs<D>, dim3(nb), dim3(kBlk), 0, st, g, mom, S.l.p);
  hipLaunchKernelGGL(k_fine_jacobi<D>, dim3(nb), dim3(kBlk), 0, st, g, S.K.p, S.Dinv.p, d_status);
  if (hipGetLastError() != hipSuccess) return LRBMS_E_HIP;
  int rc;
  if (!S.have_mg && (rc = build_hierarchy<D>(S))) return rc;
  // damping of the level-0 smoother from a power estimate of lambda_max(D^-1 A)
  std::vector<double> h(nbc);
  double* v = S.z.p;
  double* w = S.Ap.p;
  hipLaunchKernelGGL(k_power_start, dim3(blocks_for((long long)n)), dim3(kBlk), 0, st,
                     (long long)n, v);
  double scale = 1.0, lam = 0.0;
  for (int k = 0; k < 12; ++k) {
    hipLaunchKernelGGL(k_power<D>, dim3(nbc), dim3(kBlk), 0, st, g, S.K.p, S.Dinv.p, v, scale, w,
                       S.prr.p);
    if (hipMemcpy(h.data(), S.prr.p, nbc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return LRBMS_E_HIP;
    const double nrm = std::sqrt(host_sum(h));
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return LRBMS_E_NONFINITE;
    if (k > 0) lam = nrm;   // |D^-1 A v| for a unit v
    scale = 1.0 / nrm;
    std::swap(v, w);
  }
  const double omega0 = kMgOmega0 / lam;
  // conjugate gradients
  if (warm)
    hipLaunchKernelGGL((k_cg_init<D, true>), dim3(nbc), dim3(kBlk), 0, st, g, S.K.p, S.l.p, d_p,
                       S.r.p, S.prr.p, S.ppap.p);
  else
    hipLaunchKernelGGL((k_cg_init<D, false>), dim3(nbc), dim3(kBlk), 0, st, g, S.K.p, S.l.p, d_p,
                       S.r.p, S.prr.p, S.ppap.p);
  if (hipMemcpy(h.data(), S.prr.p, nbc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return LRBMS_E_HIP;
  double rr = host_sum(h);
  if (hipMemcpy(h.data(), S.ppap.p, nbc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return LRBMS_E_HIP;
  const double bb = host_sum(h);
  if (!std::isfinite(rr)) return LRBMS_E_NONFINITE;
  bool conv = !(rr > rtol * rtol * bb);   // zero right-hand side or a converged start
  int it = 0;
  if (!conv) {
    vcycle<D>(S, omega0, S.r.p, S.z.p, S.prz.p);
    hipLaunchKernelGGL((k_cg_direction<D, true>), dim3(nbc), dim3(kBlk), 0, st, g, S.K.p, S.z.p,
                       S.pv.p, S.Ap.p, S.prz.p, S.prz.p, S.ppap.p);
  }
  for (; it < maxit && !conv; ++it) {
    double* cur = S.prz.p + (size_t)(it & 1) * nbc;
    double* nxt = S.prz.p + (size_t)((it + 1) & 1) * nbc;
    hipLaunchKernelGGL(k_cg_update<D>, dim3(nbc), dim3(kBlk), 0, st, g, d_p, S.r.p, S.pv.p,
                       S.Ap.p, cur, S.ppap.p, S.prr.p, d_fail);
    if ((it + 1) % 5 == 0 || it + 1 == maxit) {
      int f = 0;
      if (hipMemcpy(h.data(), S.prr.p, nbc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(&f, d_fail, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return LRBMS_E_HIP;
      if (f) return LRBMS_E_NOT_SPD;
      rr = host_sum(h);
      if (!std::isfinite(rr)) return LRBMS_E_NONFINITE;
      conv = !(rr > rtol * rtol * bb);
      if (conv) {
        ++it;
        break;
      }
    }
    vcycle<D>(S, omega0, S.r.p, S.z.p, nxt);
    hipLaunchKernelGGL((k_cg_direction<D, false>), dim3(nbc), dim3(kBlk), 0, st, g, S.K.p, S.z.p,
                       S.pv.p, S.Ap.p, nxt, cur, S.ppap.p);
  }
  if (hipDeviceSynchronize() != hipSuccess || hipGetLastError() != hipSuccess) return LRBMS_E_HIP;
  if (iters) *iters = it;
  if (relres) *relres = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
  return conv ? LRBMS_OK : LRBMS_E_STATE;
}

FineSolver* fine_solver_create(const Geom& g) {
  std::unique_ptr<FineSolver> S(new FineSolver());
  S->g = g;
  const int D = g.dim, R = D + 1, nc = g.ncell;
  const size_t n = (size_t)R * nc;
  S->nb = blocks_for(nc);
  S->nbc = std::min(S->nb, kCgMaxBlocks);
  if (!S->K.alloc((size_t)(1 + 2 * D) * R * R * nc) || !S->Dinv.alloc((size_t)R * R * nc) ||
      !S->l.alloc(n) || !S->r.alloc(n) || !S->z.alloc(n) || !S->pv.alloc(n) || !S->Ap.alloc(n) ||
      !S->prz.alloc(2 * (size_t)S->nbc) || !S->prr.alloc(S->nbc) || !S->ppap.alloc(S->nbc) ||
      !S->fl.alloc(1))
    return nullptr;
  return S.release();
}

void fine_solver_destroy(FineSolver* S) { delete S; }

// The operator b_h(., .; gamma) of a mobility field, kept for energy norms.
template <int D>
static int energy_setup_t(FineSolver& S, double* mom, const double* field) {
  constexpr int R = D + 1;
  const Geom& g = S.g;
  const int nc = g.ncell;
  if (!S.Kbar.alloc((size_t)(1 + 2 * D) * R * R * nc) || !S.ework.alloc((size_t)R * nc))
    return LRBMS_E_OOM;
  if (launch_moments(g, field, GAMMA_FIELD, nullptr, 0, 0, mom, 0) != hipSuccess) return LRBMS_E_HIP;
  hipLaunchKernelGGL(k_fine_stencil<D>, dim3(blocks_for((long long)nc * R)), dim3(kBlk), 0, 0, g,
                     mom, S.Kbar.p);
  if (hipGetLastError() != hipSuccess) return LRBMS_E_HIP;
  S.have_bar = true;
  return LRBMS_OK;
}

int fine_energy_setup(FineSolver* S, double* mom, const double* field) {
  return S->g.dim == 2 ? energy_setup_t<2>(*S, mom, field) : energy_setup_t<3>(*S, mom, field);
}

// |a - b|^2 in the energy norm of the kept operator (a, b device fields).
int fine_energy_diff(FineSolver* S, const double* a, const double* b, double* out) {
  if (!S->have_bar) return LRBMS_E_STATE;
  const Geom& g = S->g;
  const long long n = (long long)g.r * g.ncell;
  double* e = S->ework.p;
  if (b) {
    hipLaunchKernelGGL(k_diff, dim3(blocks_for(n)), dim3(kBlk), 0, 0, n, a, b, e);
  } else if (hipMemcpy(e, a, n * sizeof(double), hipMemcpyDeviceToDevice) != hipSuccess) {
    return LRBMS_E_HIP;
  }
  if (g.dim == 2)
    hipLaunchKernelGGL(k_energy<2>, dim3(S->nbc), dim3(kBlk), 0, 0, g, S->Kbar.p, e, S->prr.p);
  else
    hipLaunchKernelGGL(k_energy<3>, dim3(S->nbc), dim3(kBlk), 0, 0, g, S->Kbar.p, e, S->prr.p);
  std::vector<double> h(S->nbc);
  if (hipMemcpy(h.data(), S->prr.p, S->nbc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return LRBMS_E_HIP;
  *out = host_sum(h);
  return std::isfinite(*out) ? LRBMS_OK : LRBMS_E_NONFINITE;
}

// |a_i - b_i|^2 (b nullable) for n pairs a_i = a + i as, b_i = b + i bs: the
// kernels of fine_energy_diff per pair, the partial sums of all pairs read
// back at once and summed on the host in the same order.
int fine_energy_diff_batch(FineSolver* S, const double* a, long long as, const double* b,
                           long long bs, int n, double* out) {
  if (!S->have_bar) return LRBMS_E_STATE;
  if (n <= 0) return LRBMS_OK;
  const Geom& g = S->g;
  const long long len = (long long)g.r * g.ncell;
  double* e = S->ework.p;
  double* parts = nullptr;
  if (hipMalloc(&parts, (size_t)n * S->nbc * sizeof(double)) != hipSuccess) return LRBMS_E_OOM;
  for (int i = 0; i < n; ++i) {
    const double* ai = a + (long long)i * as;
    if (b) {
      hipLaunchKernelGGL(k_diff, dim3(blocks_for(len)), dim3(kBlk), 0, 0, len, ai,
                         b + (long long)i * bs, e);
    } else if (hipMemcpyAsync(e, ai, len * sizeof(double), hipMemcpyDeviceToDevice, 0) !=
               hipSuccess) {
      (void)hipFree(parts);
      return LRBMS_E_HIP;
    }
    double* pr = parts + (size_t)i * S->nbc;
    if (g.dim == 2)
      hipLaunchKernelGGL(k_energy<2>, dim3(S->nbc), dim3(kBlk), 0, 0, g, S->Kbar.p, e, pr);
    else
      hipLaunchKernelGGL(k_energy<3>, dim3(S->nbc), dim3(kBlk), 0, 0, g, S->Kbar.p, e, pr);
  }
  std::vector<double> h((size_t)n * S->nbc);
  const hipError_t err = hipMemcpy(h.data(), parts, h.size() * sizeof(double),
                                   hipMemcpyDeviceToHost);
  (void)hipFree(parts);
  if (err != hipSuccess) return LRBMS_E_HIP;
  for (int i = 0; i < n; ++i) {
    out[i] = host_sum(std::vector<double>(h.begin() + (size_t)i * S->nbc,
                                          h.begin() + (size_t)(i + 1) * S->nbc));
    if (!std::isfinite(out[i])) return LRBMS_E_NONFINITE;
  }
  return LRBMS_OK;
}

int fine_solver_solve(FineSolver* S, double* mom, const double* field, int kind, double rtol,
                      int maxit, bool warm, double* d_p, int* d_status, int* iters,
                      double* relres) {
  return S->g.dim == 2 ? fine_solve_t<2>(*S, mom, field, kind, rtol, maxit, warm, d_p, d_status,
                                         iters, relres)
                       : fine_solve_t<3>(*S, mom, field, kind, rtol, maxit, warm, d_p, d_status,
                                         iters, relres);
}

// Largest entries of two partial arrays (one workgroup): out[0] = max a,
// out[1] = max b; a NaN anywhere gives NaN.
__global__ __launch_bounds__(kBlk) void k_max_pair(const double* __restrict__ a,
                                                   const double* __restrict__ b, int n,
                                                   double* __restrict__ out) {
  __shared__ double ra[kBlk], rb[kBlk];
  double ma = 0.0, mb = 0.0;
  bool nan = false;
  for (int i = threadIdx.x; i < n; i += kBlk) {
    const double x = a[i], y = b[i];
    nan = nan || x != x || y != y;
    ma = fmax(ma, x);
    mb = fmax(mb, y);
  }
  ra[threadIdx.x] = nan ? NAN : ma;
  rb[threadIdx.x] = mb;
  __syncthreads();
  if (threadIdx.x == 0) {
    double xa = 0.0, xb = 0.0;
    bool bad = false;
    for (int i = 0; i < kBlk; ++i) {
      bad = bad || ra[i] != ra[i];
      xa = fmax(xa, ra[i]);
      xb = fmax(xb, rb[i]);
    }
    out[0] = bad ? NAN : xa;
    out[1] = xb;
  }
}

size_t tof_scratch_doubles(const Geom& g) {
  const size_t R = g.dim + 1, nc = g.ncell, nb = (nc + kBlk - 1) / kBlk;
  return R * R * nc + 2 * g.dim * R * R * nc + 2 * R * nc + 2 * nb + 2;
}

void tof_carve(const Geom& g, double* base, TofBufs& B) {
  const size_t R = g.dim + 1, nc = g.ncell, nb = (nc + kBlk - 1) / kBlk;
  B.Minv = base;
  B.C = B.Minv + R * R * nc;
  B.b = B.C + 2 * g.dim * R * R * nc;
  B.other = B.b + R * nc;
  B.pc = B.other + R * nc;
  B.ps = B.pc + nb;
  B.red = B.ps + nb;
}

// The sweeps on given work buffers (no allocation): set-up of the cell
// blocks, then block-Jacobi sweeps; every 16 sweeps the largest change and
// the largest coefficient come back to the host (two doubles).
template <int D>
static int tof_solve_t(const Geom& g, const double* d_flux, double tol, int maxit, double* d_tau,
                       int* d_status, int* sweeps, const TofBufs& B) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  const size_t n = (size_t)R * nc;
  const int nb = blocks_for(nc);
  hipStream_t st = 0;
  hipLaunchKernelGGL(k_tof_setup<D>, dim3(nb), dim3(kBlk), 0, st, g, d_flux, B.Minv, B.C, B.b,
                     d_status);
  if (hipMemsetAsync(d_tau, 0, n * sizeof(double), st) != hipSuccess) return LRBMS_E_HIP;
  double* cur = d_tau;
  double* nxt = B.other;
  int it = 0;
  bool done = false;
  for (; it < maxit && !done; ++it) {
    hipLaunchKernelGGL(k_tof_sweep<D>, dim3(nb), dim3(kBlk), 0, st, g, B.Minv, B.C, B.b, cur, nxt,
                       B.pc, B.ps);
    std::swap(cur, nxt);
    if ((it + 1) % 16 == 0 || it + 1 == maxit) {
      hipLaunchKernelGGL(k_max_pair, dim3(1), dim3(kBlk), 0, st, B.pc, B.ps, nb, B.red);
      double h[2];
      if (hipMemcpy(h, B.red, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return LRBMS_E_HIP;
      if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return LRBMS_E_NONFINITE;
      done = h[0] <= tol * h[1];
    }
  }
  if (cur != d_tau &&
      hipMemcpy(d_tau, cur, n * sizeof(double), hipMemcpyDeviceToDevice) != hipSuccess)
    return LRBMS_E_HIP;
  if (sweeps) *sweeps = it;
  if (hipGetLastError() != hipSuccess) return LRBMS_E_HIP;
  return done ? LRBMS_OK : LRBMS_E_STATE;
}

int tof_solve_bufs(const Geom& g, const double* d_flux, double tol, int maxit, double* d_tau,
                   int* d_status, int* sweeps, const TofBufs& B) {
  return g.dim == 2 ? tof_solve_t<2>(g, d_flux, tol, maxit, d_tau, d_status, sweeps, B)
                    : tof_solve_t<3>(g, d_flux, tol, maxit, d_tau, d_status, sweeps, B);
}

int tof_solve(const Geom& g, const double* d_flux, double tol, int maxit, double* d_tau,
              int* d_status, int* sweeps) {
  DevBuf work;
  if (!work.alloc(tof_scratch_doubles(g))) return LRBMS_E_OOM;
  TofBufs B;
  tof_carve(g, work.p, B);
  return tof_solve_bufs(g, d_flux, tol, maxit, d_tau, d_status, sweeps, B);
}

}  // namespace lrbms
