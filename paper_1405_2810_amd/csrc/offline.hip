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

// ---- preconditioned conjugate gradients, two launches per iteration ----------
// The scalars never leave the device: every workgroup sums the per-workgroup
// partials of the previous launch itself, in the same fixed order, so all
// workgroups see identical alpha and beta.  Ap is carried by the recursion
// A p_new = A z + beta A p_old, so one operator application per iteration
// serves both the search direction and the curvature p . Ap.  The grid is
// capped (grid-stride loops) to bound the partial sums.
constexpr int kCgMaxBlocks = 1024;

__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlk) s += p[i];
  return block_sum(s, red);
}

// Apply the cell's r x r blocks to v (own and face neighbours' coefficients).
template <int D>
__device__ __forceinline__ void stencil_apply(const Geom& g, const double* __restrict__ K,
                                              const double* __restrict__ v, int c,
                                              double (&y)[D + 1]) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  int xc[3];
  cell_coords(g, c, xc);
  double u[1 + 2 * D][R];
#pragma unroll
  for (int k = 0; k < R; ++k) u[0][k] = v[(size_t)k * nc + c];
#pragma unroll
  for (int f = 0; f < 2 * D; ++f) {
    const int n = face_neighbour(g, xc, f);
#pragma unroll
    for (int k = 0; k < R; ++k) u[1 + f][k] = (n >= 0) ? v[(size_t)k * nc + n] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    double s = 0.0;
#pragma unroll
    for (int f = 0; f < 1 + 2 * D; ++f)
#pragma unroll
      for (int kp = 0; kp < R; ++kp) s = fma(K[(size_t)((f * R + k) * R + kp) * nc + c], u[f][kp], s);
    y[k] = s;
  }
}

// x = 0, r = b, z = D^-1 b; partials of r.z and r.r.
template <int D>
__global__ __launch_bounds__(kBlk) void k_cg_init(Geom g, const double* __restrict__ b,
                                                  const double* __restrict__ Dinv,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ z,
                                                  double* __restrict__ part_rz,
                                                  double* __restrict__ part_rr) {
  constexpr int R = D + 1;
  __shared__ double red[4];
  const int nc = g.ncell;
  double rz = 0.0, rr = 0.0;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += gridDim.x * kBlk) {
    double rv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rv[k] = b[(size_t)k * nc + c];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) t = fma(Dinv[(size_t)(i * R + j) * nc + c], rv[j], t);
      x[(size_t)i * nc + c] = 0.0;
      r[(size_t)i * nc + c] = rv[i];
      z[(size_t)i * nc + c] = t;
      rz = fma(rv[i], t, rz);
      rr = fma(rv[i], rv[i], rr);
    }
  }
  const double a = block_sum(rz, red);
  const double bb = block_sum(rr, red);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = a;
    part_rr[blockIdx.x] = bb;
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
    double w[R];
    stencil_apply<D>(g, K, z, c, w);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const size_t i = (size_t)k * nc + c;
      const double pk = FIRST ? z[i] : fma(beta, p[i], z[i]);
      const double ak = FIRST ? w[k] : fma(beta, Ap[i], w[k]);
      p[i] = pk;
      Ap[i] = ak;
      dot = fma(pk, ak, dot);
    }
  }
  const double t = block_sum(dot, red);
  if (threadIdx.x == 0) part_pap[blockIdx.x] = t;
}

// alpha = (r.z) / (p.Ap); x += alpha p, r -= alpha Ap, z = D^-1 r; partials
// of the new r.z and r.r.  A non-positive or non-finite curvature sets fail.
template <int D>
__global__ __launch_bounds__(kBlk) void k_cg_update(Geom g, const double* __restrict__ Dinv,
                                                    double* __restrict__ x, double* __restrict__ r,
                                                    double* __restrict__ z,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ Ap,
                                                    const double* __restrict__ rz_cur,
                                                    const double* __restrict__ part_pap,
                                                    double* __restrict__ rz_next,
                                                    double* __restrict__ part_rr,
                                                    int* __restrict__ fail) {
  constexpr int R = D + 1;
  __shared__ double red[4];
  const int nc = g.ncell, nb = gridDim.x;
  const double rz = sum_partials(rz_cur, nb, red);
  const double pap = sum_partials(part_pap, nb, red);
  const bool ok = pap > 0.0 && isfinite(pap);
  const double al = ok ? rz / pap : 0.0;
  if (!ok && blockIdx.x == 0 && threadIdx.x == 0) *fail = 1;
  double rzn = 0.0, rr = 0.0;
  for (int c = blockIdx.x * kBlk + threadIdx.x; c < nc; c += nb * kBlk) {
    double rv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const size_t i = (size_t)k * nc + c;
      x[i] = fma(al, p[i], x[i]);
      rv[k] = fma(-al, Ap[i], r[i]);
      r[i] = rv[k];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) t = fma(Dinv[(size_t)(i * R + j) * nc + c], rv[j], t);
      z[(size_t)i * nc + c] = t;
      rzn = fma(rv[i], t, rzn);
      rr = fma(rv[i], rv[i], rr);
    }
  }
  const double a = block_sum(rzn, red);
  const double bb = block_sum(rr, red);
  if (threadIdx.x == 0) {
    rz_next[blockIdx.x] = a;
    part_rr[blockIdx.x] = bb;
  }
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
  bool alloc(size_t n) { return hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(double)) == hipSuccess; }
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

template <int D>
static int fine_solve_t(const Geom& g, double* mom, const double* field, int kind, double rtol,
                        int maxit, double* d_p, int* d_status, int* iters, double* relres) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  const size_t n = (size_t)R * nc;
  const int nb = blocks_for(nc);
  const int nbc = std::min(nb, kCgMaxBlocks);
  hipStream_t st = 0;
  DevBuf K, Dinv, l, r, z, pv, Ap, prz, prr, ppap, fl;
  if (!K.alloc((size_t)(1 + 2 * D) * R * R * nc) || !Dinv.alloc((size_t)R * R * nc) ||
      !l.alloc(n) || !r.alloc(n) || !z.alloc(n) || !pv.alloc(n) || !Ap.alloc(n) ||
      !prz.alloc(2 * (size_t)nbc) || !prr.alloc(nbc) || !ppap.alloc(nbc) || !fl.alloc(1))
    return LRBMS_E_OOM;
  int* d_fail = reinterpret_cast<int*>(fl.p);
  if (hipMemset(d_fail, 0, sizeof(int)) != hipSuccess) return LRBMS_E_HIP;
  if (launch_moments(g, field, kind, nullptr, 0, 0, mom, st) != hipSuccess) return LRBMS_E_HIP;
  hipLaunchKernelGGL(k_fine_stencil<D>, dim3(blocks_for((long long)nc * R)), dim3(kBlk), 0, st, g,
                     mom, K.p);
  hipLaunchKernelGGL(k_fine_rhs<D>, dim3(nb), dim3(kBlk), 0, st, g, mom, l.p);
  hipLaunchKernelGGL(k_fine_jacobi<D>, dim3(nb), dim3(kBlk), 0, st, g, K.p, Dinv.p, d_status);
  hipLaunchKernelGGL(k_cg_init<D>, dim3(nbc), dim3(kBlk), 0, st, g, l.p, Dinv.p, d_p, r.p, z.p,
                     prz.p, prr.p);
  hipLaunchKernelGGL((k_cg_direction<D, true>), dim3(nbc), dim3(kBlk), 0, st, g, K.p, z.p, pv.p,
                     Ap.p, prz.p, prz.p, ppap.p);
  if (hipGetLastError() != hipSuccess) return LRBMS_E_HIP;
  std::vector<double> h(nbc);
  if (hipMemcpy(h.data(), prr.p, nbc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return LRBMS_E_HIP;
  const double bb = host_sum(h);
  double rr = bb;
  bool conv = !(rr > rtol * rtol * bb);   // zero right-hand side
  int it = 0;
  for (; it < maxit && !conv; ++it) {
    double* cur = prz.p + (size_t)(it & 1) * nbc;
    double* nxt = prz.p + (size_t)((it + 1) & 1) * nbc;
    hipLaunchKernelGGL(k_cg_update<D>, dim3(nbc), dim3(kBlk), 0, st, g, Dinv.p, d_p, r.p, z.p,
                       pv.p, Ap.p, cur, ppap.p, nxt, prr.p, d_fail);
    const bool check = (it + 1) % 20 == 0 || it + 1 == maxit;
    if (check) {
      int f = 0;
      if (hipMemcpy(h.data(), prr.p, nbc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
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
    hipLaunchKernelGGL((k_cg_direction<D, false>), dim3(nbc), dim3(kBlk), 0, st, g, K.p, z.p,
                       pv.p, Ap.p, nxt, cur, ppap.p);
  }
  if (hipDeviceSynchronize() != hipSuccess || hipGetLastError() != hipSuccess) return LRBMS_E_HIP;
  if (iters) *iters = it;
  if (relres) *relres = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
  return conv ? LRBMS_OK : LRBMS_E_STATE;
}

int fine_solve(const Geom& g, double* mom, const double* field, int kind, double rtol, int maxit,
               double* d_p, int* d_status, int* iters, double* relres) {
  return g.dim == 2 ? fine_solve_t<2>(g, mom, field, kind, rtol, maxit, d_p, d_status, iters, relres)
                    : fine_solve_t<3>(g, mom, field, kind, rtol, maxit, d_p, d_status, iters, relres);
}

template <int D>
static int tof_solve_t(const Geom& g, const double* d_flux, double tol, int maxit, double* d_tau,
                       int* d_status, int* sweeps) {
  constexpr int R = D + 1;
  const int nc = g.ncell;
  const size_t n = (size_t)R * nc;
  const int nb = blocks_for(nc);
  hipStream_t st = 0;
  DevBuf Minv, C, b, other, pc, ps;
  if (!Minv.alloc((size_t)R * R * nc) || !C.alloc((size_t)2 * D * R * R * nc) || !b.alloc(n) ||
      !other.alloc(n) || !pc.alloc(nb) || !ps.alloc(nb))
    return LRBMS_E_OOM;
  hipLaunchKernelGGL(k_tof_setup<D>, dim3(nb), dim3(kBlk), 0, st, g, d_flux, Minv.p, C.p, b.p,
                     d_status);
  if (hipMemsetAsync(d_tau, 0, n * sizeof(double), st) != hipSuccess) return LRBMS_E_HIP;
  double* cur = d_tau;
  double* nxt = other.p;
  std::vector<double> hc(nb), hs(nb);
  int it = 0;
  bool done = false;
  for (; it < maxit && !done; ++it) {
    hipLaunchKernelGGL(k_tof_sweep<D>, dim3(nb), dim3(kBlk), 0, st, g, Minv.p, C.p, b.p, cur, nxt,
                       pc.p, ps.p);
    std::swap(cur, nxt);
    if ((it + 1) % 16 == 0 || it + 1 == maxit) {
      if (hipMemcpy(hc.data(), pc.p, nb * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hs.data(), ps.p, nb * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return LRBMS_E_HIP;
      double mc = 0.0, ms = 0.0;
      for (int i = 0; i < nb; ++i) {
        mc = std::max(mc, hc[i]);
        ms = std::max(ms, hs[i]);
      }
      if (!std::isfinite(mc) || !std::isfinite(ms)) return LRBMS_E_NONFINITE;
      done = mc <= tol * ms;
    }
  }
  if (cur != d_tau &&
      hipMemcpy(d_tau, cur, n * sizeof(double), hipMemcpyDeviceToDevice) != hipSuccess)
    return LRBMS_E_HIP;
  if (sweeps) *sweeps = it;
  if (hipGetLastError() != hipSuccess) return LRBMS_E_HIP;
  return done ? LRBMS_OK : LRBMS_E_STATE;
}

int tof_solve(const Geom& g, const double* d_flux, double tol, int maxit, double* d_tau,
              int* d_status, int* sweeps) {
  return g.dim == 2 ? tof_solve_t<2>(g, d_flux, tol, maxit, d_tau, d_status, sweeps)
                    : tof_solve_t<3>(g, d_flux, tol, maxit, d_tau, d_status, sweeps);
}

}  // namespace lrbms
