// Reduced assembly on gfx950.
//
// Mobility moments (a1), the Galerkin projection A_N = Phi^T A(gamma) Phi and
// f_N = Phi^T l(gamma) of the SWIP forms of Sec. 3.2 onto the broken reduced
// space W_N (Def. coarseScalePressure), the affine sum of eq. reducedSystem
// and the least-squares fit of eq. leastSquaresFit.
//
// Readings of the printed forms used throughout (same as the CPU reference):
// consistency terms with a minus sign, Neumann term -int v_N w, SWIP mean
// weights (or the literal ones on request), two-valued mobility on faces
// (each side of the weighted mean uses its own trace), outward normal and
// weight 1 on Dirichlet faces, h_f = face diameter, zero gravity.
//
// Kernel structure: one workgroup per coarse box builds Y = K_E Phi_E a
// chunk of cells at a time (threads over (cell, column), coalesced reads of
// the column-major Phi_E, the 2d-face stencil evaluated from per-cell
// mobility moments), stages the chunk of Phi_E and Y in LDS and contracts
// Phi_E^T Y with one output column per thread.  The right-hand side rides
// along as column N_E.  One workgroup per coarse interface builds the
// coupling block the same way from the fine faces on the interface.
#include <algorithm>

#include "common.h"
#include "ktimer.h"

namespace lrbms {

// ---------------------------------------------------------------------------
// a1: mobility moments per cell.  gamma is lambda(s_h) (kind GAMMA_SAT), a P1
// field (GAMMA_FIELD) or sum_q theta_q Lambda^q (GAMMA_COMBO); integrals by the
// 2-point Gauss rules, which are exact for the quadratic mobility of a P1 state.
__global__ __launch_bounds__(256) void k_moments(Geom g, const double* __restrict__ src, int kind,
                                                 const double* __restrict__ theta, int nprof,
                                                 long long pstride, double* __restrict__ mom) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int d = g.dim, nc = g.ncell;
  double co[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < g.r; ++k) {
    if (kind == GAMMA_COMBO) {
      double v = 0.0;
      for (int q = 0; q < nprof; ++q) v += theta[q] * src[q * pstride + (long long)k * nc + c];
      co[k] = v;
    } else {
      co[k] = src[(long long)k * nc + c];
    }
  }
  // value of gamma at local point xi (sq holds sqrt(3) xi_a)
  auto gam = [&](const double sq[3]) {
    double v = co[0];
    for (int a = 0; a < d; ++a) v += sq[a] * co[a + 1];
    v *= g.isv;
    return kind == GAMMA_SAT ? total_mobility(g, v) : v;
  };
  const double gp = 1.0 / kSqrt3;
  double sq[3];
  double sum = 0.0;
  const int nq = 1 << d;
  for (int p = 0; p < nq; ++p) {
    for (int a = 0; a < d; ++a) sq[a] = kSqrt3 * (((p >> a) & 1) ? gp : -gp);
    sum += gam(sq);
  }
  mom[c] = sum * g.vol / nq;
  for (int a = 0; a < d; ++a) {
    int tax[2], nt = 0;
    for (int b = 0; b < d; ++b)
      if (b != a) tax[nt++] = b;
    const double w = g.area[a] / (1 << nt);
    for (int dir = 0; dir < 2; ++dir) {
      double m0 = 0.0, mt[2] = {0.0, 0.0};
      for (int p = 0; p < (1 << nt); ++p) {
        double xi[3] = {0.0, 0.0, 0.0};
        xi[a] = dir ? 1.0 : -1.0;
        for (int ti = 0; ti < nt; ++ti) xi[tax[ti]] = ((p >> ti) & 1) ? gp : -gp;
        for (int b = 0; b < d; ++b) sq[b] = kSqrt3 * xi[b];
        const double v = gam(sq);
        m0 += v;
        for (int ti = 0; ti < nt; ++ti) mt[ti] += v * xi[tax[ti]];
      }
      const int s = mom_slot(d, a, dir);
      mom[(long long)s * nc + c] = m0 * w;
      for (int ti = 0; ti < nt; ++ti) mom[(long long)(s + 1 + ti) * nc + c] = mt[ti] * w;
    }
  }
}

hipError_t launch_moments(const Geom& g, const double* src, int kind, const double* theta,
                          int nprof, long long prof_stride, double* mom, hipStream_t st) {
  const int nb = (g.ncell + 255) / 256;
  ktimer_begin(KK_MOMENTS, st);
  hipLaunchKernelGGL(k_moments, dim3(nb), dim3(256), 0, st, g, src, kind, theta, nprof,
                     prof_stride, mom);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Face terms of b_h for one face of a test cell and one trial column.
//   alpha = +1: the face is on the +a side of the test cell (test cell is the
//   low-side cell e1), -1: on the -a side.  On a boundary face alpha is also
//   the sign of the outward normal.  ps / po: trial coefficients on the test
//   side / the other side (zero when the trial function vanishes there).
//   ms / mo: moments of gamma on the face from the test side / other side
//   (m0 = int_f gamma, mt = int_f gamma xi_t).
// Adds to Y[k] = sum over trial dofs of the face matrix entries (row = test
// dof k of the test cell).
struct FaceCtx {
  int a;
  double alpha;
  bool interior;
  double ks, ko;
  double ms[3], mo[3];
};

__device__ __forceinline__ void face_rows(const Geom& g, const FaceCtx& f, const double* ps,
                                          const double* po, bool gam, bool pen, double* Y) {
  const int a = f.a, d = g.dim;
  const double isv = g.isv;
  const double gf = kSqrt3 * 2.0 / g.h[a] * isv;
  const double as = f.alpha, ao = -f.alpha;
  double js, jo, ws, wo, sig, nd;
  if (f.interior) {
    js = f.alpha;
    jo = -f.alpha;
    const double klo = f.alpha > 0 ? f.ks : f.ko, khi = f.alpha > 0 ? f.ko : f.ks;
    double wlo, whi;
    if (g.weights == 0) {
      wlo = khi / (klo + khi);
      whi = klo / (klo + khi);
    } else {
      wlo = klo / (klo + khi);
      whi = khi / (klo + khi);
    }
    ws = f.alpha > 0 ? wlo : whi;
    wo = f.alpha > 0 ? whi : wlo;
    sig = g.pen * 2.0 * klo * khi / (klo + khi);
    nd = gf;
  } else {
    js = 1.0;
    jo = 0.0;
    ws = 1.0;
    wo = 0.0;
    sig = g.pen * f.ks;
    nd = f.alpha * gf;
  }
  int tax[2], nt = 0;
  for (int b = 0; b < d; ++b)
    if (b != a) tax[nt++] = b;
  if (gam) {
    // -int {gamma kappa d_n v} [w]: trial normal derivatives against the test trace
    const double cs = ws * f.ks * nd * ps[a + 1];
    const double cq = f.interior ? wo * f.ko * nd * po[a + 1] : 0.0;
    const double A0 = cs * f.ms[0] + (f.interior ? cq * f.mo[0] : 0.0);
    Y[0] -= js * isv * A0;
    Y[a + 1] -= js * isv * kSqrt3 * as * A0;
    for (int ti = 0; ti < nt; ++ti) {
      const double At = cs * f.ms[1 + ti] + (f.interior ? cq * f.mo[1 + ti] : 0.0);
      Y[tax[ti] + 1] -= js * isv * kSqrt3 * At;
    }
    // -int {gamma kappa d_n w} [v]: test normal derivative against the trial jump
    double jm = js * (ps[0] * f.ms[0] + kSqrt3 * as * ps[a + 1] * f.ms[0]);
    for (int ti = 0; ti < nt; ++ti) jm += js * kSqrt3 * ps[tax[ti] + 1] * f.ms[1 + ti];
    if (f.interior) {
      jm += jo * (po[0] * f.ms[0] + kSqrt3 * ao * po[a + 1] * f.ms[0]);
      for (int ti = 0; ti < nt; ++ti) jm += jo * kSqrt3 * po[tax[ti] + 1] * f.ms[1 + ti];
    }
    Y[a + 1] -= ws * f.ks * nd * isv * jm;
  }
  if (pen) {
    // sigma_f / h_f int [v][w]
    const double P = sig / g.hf[a] * (isv * isv) * g.area[a] * js;
    double J0 = js * (ps[0] + kSqrt3 * as * ps[a + 1]);
    if (f.interior) J0 += jo * (po[0] + kSqrt3 * ao * po[a + 1]);
    Y[0] += P * J0;
    Y[a + 1] += P * kSqrt3 * as * J0;
    for (int ti = 0; ti < nt; ++ti) {
      const int t = tax[ti] + 1;
      Y[t] += P * (js * ps[t] + (f.interior ? jo * po[t] : 0.0));
    }
  }
}

__device__ __forceinline__ void load_moments(const Geom& g, const double* mom, int c, int a,
                                             int dir, double* m) {
  const int s = mom_slot(g.dim, a, dir);
  for (int q = 0; q < g.dim; ++q) m[q] = mom[(long long)(s + q) * g.ncell + c];
}

// Rows (e, 0..r-1) of K_E Phi for one column of Phi^E (test cell e at box-local
// index l, box coordinates x).  Trial values outside the box are zero.
__device__ void cell_rows(const Geom& g, const Sub& S, int e, const int x[3], int l,
                          const double* __restrict__ col, const double* ps,
                          const double* __restrict__ mom, int parts, double* Y) {
  const int d = g.dim, r = g.r;
  const bool gam = parts & PART_GAMMA, pen = parts & PART_PEN;
  const double ke = g.perm[e];
  if (gam) {
    const double mv = mom[e];
    for (int a = 0; a < d; ++a) {
      const double gf = kSqrt3 * 2.0 / g.h[a] * g.isv;
      Y[a + 1] += ke * mv * (gf * gf) * ps[a + 1];
    }
  }
  int bstride[3] = {1, S.hi[0] - S.lo[0], (S.hi[0] - S.lo[0]) * (S.hi[1] - S.lo[1])};
  for (int a = 0; a < d; ++a) {
    for (int dir = 0; dir < 2; ++dir) {
      FaceCtx f;
      f.a = a;
      f.alpha = dir ? 1.0 : -1.0;
      f.ks = ke;
      load_moments(g, mom, e, a, dir, f.ms);
      int xn[3] = {x[0], x[1], x[2]};
      xn[a] += dir ? 1 : -1;
      double po[4] = {0.0, 0.0, 0.0, 0.0};
      if (xn[a] >= 0 && xn[a] < g.n[a]) {
        const int en = cell_index(g, xn);
        f.interior = true;
        f.ko = g.perm[en];
        load_moments(g, mom, en, a, 1 - dir, f.mo);
        if (xn[a] >= S.lo[a] && xn[a] < S.hi[a]) {
          const int ln = l + (dir ? bstride[a] : -bstride[a]);
          for (int k = 0; k < r; ++k) po[k] = col[(long long)k * S.nE + ln];
        }
        face_rows(g, f, ps, po, gam, pen, Y);
      } else {
        int xf[3] = {x[0], x[1], x[2]};
        xf[a] += dir;
        const int fid = face_index(g, a, xf);
        if (g.bc_type[fid] == LRBMS_BC_DIRICHLET) {
          f.interior = false;
          f.ko = 0.0;
          face_rows(g, f, ps, po, gam, pen, Y);
        }
      }
    }
  }
}

// l_h(phi_k) of test cell e (sources, Neumann and Dirichlet data).
__device__ void cell_rhs(const Geom& g, int e, const int x[3], const double* __restrict__ mom,
                         int parts, double* Y) {
  const int d = g.dim;
  if (parts & PART_RHS_CONST) Y[0] += g.q1[e] * g.vol * g.isv;
  for (int a = 0; a < d; ++a) {
    for (int dir = 0; dir < 2; ++dir) {
      int xn[3] = {x[0], x[1], x[2]};
      xn[a] += dir ? 1 : -1;
      if (xn[a] >= 0 && xn[a] < g.n[a]) continue;
      int xf[3] = {x[0], x[1], x[2]};
      xf[a] += dir;
      const int fid = face_index(g, a, xf);
      const int bt = g.bc_type[fid];
      const double val = g.bc_val[fid];
      const double al = dir ? 1.0 : -1.0;
      const double tw0 = g.area[a] * g.isv, twa = tw0 * kSqrt3 * al;   // int_f phi_0, phi_{a+1}
      if (bt == LRBMS_BC_NEUMANN && (parts & PART_RHS_CONST)) {
        Y[0] -= val * tw0;
        Y[a + 1] -= val * twa;
      } else if (bt == LRBMS_BC_DIRICHLET) {
        if (parts & PART_RHS_CONST) {
          const double sg = g.pen * g.perm[e] / g.hf[a];
          Y[0] += sg * val * tw0;
          Y[a + 1] += sg * val * twa;
        }
        if (parts & PART_RHS_GAMMA) {
          const double gf = kSqrt3 * 2.0 / g.h[a] * g.isv;
          const double m0 = mom[(long long)mom_slot(d, a, dir) * g.ncell + e];
          Y[a + 1] -= val * g.perm[e] * m0 * (al * gf);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fine SWIP operator (Def. pressureDG) without assembly, for the offline
// snapshot solves: y = A(gamma) x on every cell, the right-hand side l(gamma),
// and the inverse r x r diagonal blocks used as block-Jacobi preconditioner.
__device__ __noinline__ void fine_rows(const Geom& g, int e, const double* __restrict__ x,
                          const double* __restrict__ mom, bool with_nbr, const double* ps_in,
                          double* Y) {
  const int d = g.dim, r = g.r, nc = g.ncell;
  int xc[3];
  cell_coords(g, e, xc);
  double ps[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < r; ++k) ps[k] = ps_in ? ps_in[k] : x[(long long)k * nc + e];
  const double ke = g.perm[e];
  const double mv = mom[e];
  for (int a = 0; a < d; ++a) {
    const double gf = kSqrt3 * 2.0 / g.h[a] * g.isv;
    Y[a + 1] += ke * mv * (gf * gf) * ps[a + 1];
  }
  for (int a = 0; a < d; ++a) {
    for (int dir = 0; dir < 2; ++dir) {
      FaceCtx f;
      f.a = a;
      f.alpha = dir ? 1.0 : -1.0;
      f.ks = ke;
      load_moments(g, mom, e, a, dir, f.ms);
      int xn[3] = {xc[0], xc[1], xc[2]};
      xn[a] += dir ? 1 : -1;
      double po[4] = {0.0, 0.0, 0.0, 0.0};
      if (xn[a] >= 0 && xn[a] < g.n[a]) {
        const int en = cell_index(g, xn);
        f.interior = true;
        f.ko = g.perm[en];
        load_moments(g, mom, en, a, 1 - dir, f.mo);
        if (with_nbr)
          for (int k = 0; k < r; ++k) po[k] = x[(long long)k * nc + en];
        face_rows(g, f, ps, po, true, true, Y);
      } else {
        int xf[3] = {xc[0], xc[1], xc[2]};
        xf[a] += dir;
        if (g.bc_type[face_index(g, a, xf)] == LRBMS_BC_DIRICHLET) {
          f.interior = false;
          f.ko = 0.0;
          face_rows(g, f, ps, po, true, true, Y);
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_fine_apply(Geom g, const double* __restrict__ mom,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.ncell) return;
  double Y[4] = {0.0, 0.0, 0.0, 0.0};
  fine_rows(g, e, x, mom, true, nullptr, Y);
  for (int k = 0; k < g.r; ++k) y[(long long)k * g.ncell + e] = Y[k];
}

hipError_t launch_fine_apply(const Geom& g, const double* mom, const double* x, double* y,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_fine_apply, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g, mom, x, y);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fine_rhs(Geom g, const double* __restrict__ mom,
                                                  double* __restrict__ l) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.ncell) return;
  int xc[3];
  cell_coords(g, e, xc);
  double Y[4] = {0.0, 0.0, 0.0, 0.0};
  cell_rhs(g, e, xc, mom, PART_RHS_CONST | PART_RHS_GAMMA, Y);
  for (int k = 0; k < g.r; ++k) l[(long long)k * g.ncell + e] = Y[k];
}

hipError_t launch_fine_rhs(const Geom& g, const double* mom, double* l, hipStream_t st) {
  hipLaunchKernelGGL(k_fine_rhs, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g, mom, l);
  return hipGetLastError();
}

// Inverse of the r x r diagonal block of every cell (Gauss-Jordan, no pivoting:
// the blocks are SPD).
__global__ __launch_bounds__(256) void k_fine_jacobi(Geom g, const double* __restrict__ mom,
                                                     double* __restrict__ dinv) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.ncell) return;
  const int r = g.r;
  double D[4][8];
  for (int j = 0; j < r; ++j) {
    double unit[4] = {0.0, 0.0, 0.0, 0.0};
    unit[j] = 1.0;
    double Y[4] = {0.0, 0.0, 0.0, 0.0};
    fine_rows(g, e, nullptr, mom, false, unit, Y);
    for (int i = 0; i < r; ++i) {
      D[i][j] = Y[i];
      D[i][r + j] = (i == j) ? 1.0 : 0.0;
    }
  }
  for (int c = 0; c < r; ++c) {
    const double piv = D[c][c];
    for (int j = 0; j < 2 * r; ++j) D[c][j] /= piv;
    for (int i = 0; i < r; ++i) {
      if (i == c) continue;
      const double f = D[i][c];
      for (int j = 0; j < 2 * r; ++j) D[i][j] -= f * D[c][j];
    }
  }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) dinv[(long long)(i * r + j) * g.ncell + e] = D[i][r + j];
}

hipError_t launch_fine_jacobi(const Geom& g, const double* mom, double* dinv, hipStream_t st) {
  hipLaunchKernelGGL(k_fine_jacobi, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g, mom, dinv);
  return hipGetLastError();
}

// Diagonal blocks A[E][E] and f_E.  One workgroup per (box, chunk of cells):
//   stencil  the r x r blocks coupling each cell of the chunk to itself and to
//            its 2d face neighbours, found once per cell by applying the face
//            terms to unit trial vectors (summed over faces in a fixed order);
//   apply    Y(cell, :) = K Phi for every (cell, column) pair, coalesced reads
//            of the column-major Phi^E (neighbours outside the box are zero);
//   contract partial A_E = Phi_chunk^T Y_chunk with one output column per
//            thread; the right-hand side rides along as column N_E.
// The partial blocks are summed over the chunks of a box in a fixed order by
// k_reduce_diag.
constexpr int kChunk = 32;

__device__ void cell_stencil(const Geom& g, int e, const int x[3], const double* __restrict__ mom,
                             int parts, int m, int kp, double* out) {
  // m = 0: volume term; m = 1 + 2a + dir: face (a, dir).  Column kp of the block
  // for the own trial dofs (out[0..r)) and, on interior faces, for the
  // neighbour's trial dofs (out[r..2r)).
  const int r = g.r;
  const bool gam = parts & PART_GAMMA, pen = parts & PART_PEN;
  double unit[4] = {0.0, 0.0, 0.0, 0.0}, zero[4] = {0.0, 0.0, 0.0, 0.0};
  unit[kp] = 1.0;
  for (int k = 0; k < 2 * r; ++k) out[k] = 0.0;
  const double ke = g.perm[e];
  if (m == 0) {
    if (gam && kp >= 1) {
      const int a = kp - 1;
      const double gf = kSqrt3 * 2.0 / g.h[a] * g.isv;
      out[kp] = ke * mom[e] * (gf * gf);
    }
    return;
  }
  const int a = (m - 1) / 2, dir = (m - 1) % 2;
  FaceCtx f;
  f.a = a;
  f.alpha = dir ? 1.0 : -1.0;
  f.ks = ke;
  load_moments(g, mom, e, a, dir, f.ms);
  int xn[3] = {x[0], x[1], x[2]};
  xn[a] += dir ? 1 : -1;
  if (xn[a] >= 0 && xn[a] < g.n[a]) {
    const int en = cell_index(g, xn);
    f.interior = true;
    f.ko = g.perm[en];
    load_moments(g, mom, en, a, 1 - dir, f.mo);
    face_rows(g, f, unit, zero, gam, pen, out);
    face_rows(g, f, zero, unit, gam, pen, out + r);
  } else {
    int xf[3] = {x[0], x[1], x[2]};
    xf[a] += dir;
    if (g.bc_type[face_index(g, a, xf)] == LRBMS_BC_DIRICHLET) {
      f.interior = false;
      f.ko = 0.0;
      face_rows(g, f, unit, zero, gam, pen, out);
    }
  }
}

template <int COLS>
__host__ __device__ constexpr int chunk_cells() { return COLS <= 32 ? kChunk : kChunk / 2; }

// Dynamic LDS of the box assembly: stencil blocks, then the Phi and Y staging.
// The staging area also holds the tree reduction: (256 / cols / 2) * cols rows.
__host__ __device__ inline size_t diag_lds_doubles(int cols, int r, int d) {
  const int ch = cols <= 32 ? kChunk : kChunk / 2;
  const size_t stage = 2 * (size_t)ch * r * (cols + 1);
  const size_t red = (size_t)(256 / cols / 2) * cols * (cols + 1);
  return (size_t)ch * (1 + 2 * d) * 2 * r * r + (stage > red ? stage : red);
}

template <int COLS>
__global__ __launch_bounds__(256) void k_assemble_diag(Geom g, const Sub* __restrict__ subs,
                                                       const int* __restrict__ chunks,
                                                       const double* __restrict__ phi,
                                                       const double* __restrict__ mom, int parts,
                                                       double* __restrict__ partial) {
  constexpr int stride = COLS + 1;
  constexpr int NG = 256 / COLS;
  constexpr int CH = chunk_cells<COLS>();
  extern __shared__ double lds[];
  __shared__ int cellg[CH], cellx[CH][3], nbl[CH][6];
  const int sub = chunks[2 * blockIdx.x], c0 = chunks[2 * blockIdx.x + 1];
  const Sub S = subs[sub];
  const int NE = S.NE, nE = S.nE, r = g.r, d = g.dim, rr = r * r;
  const int nm = 1 + 2 * d;
  double* Kc = lds;                                   // [CH][nm][2][r*r]
  double* Phil = Kc + (size_t)CH * nm * 2 * rr;       // [CH][r][stride]
  double* Yl = Phil + (size_t)CH * r * stride;        // [CH][r][stride]
  auto K = [&](int lc, int m, int side, int k, int kp) -> double& {
    return Kc[(((size_t)lc * nm + m) * 2 + side) * rr + k * r + kp];
  };
  const bool want_rhs = parts & (PART_RHS_CONST | PART_RHS_GAMMA);
  const bool want_mat = parts & (PART_GAMMA | PART_PEN);
  const int ncol = NE + (want_rhs ? 1 : 0);
  const int cc = min(CH, nE - c0);
  const int bx = S.hi[0] - S.lo[0], by = S.hi[1] - S.lo[1];
  const int bstride[3] = {1, bx, bx * by};
  for (int lc = threadIdx.x; lc < cc; lc += blockDim.x) {
    const int l = c0 + lc;
    const int x[3] = {S.lo[0] + l % bx, S.lo[1] + (l / bx) % by, S.lo[2] + l / (bx * by)};
    cellg[lc] = cell_index(g, x);
    for (int q = 0; q < 3; ++q) cellx[lc][q] = x[q];
    for (int a = 0; a < 3; ++a)
      for (int dir = 0; dir < 2; ++dir) {
        const int xa = x[a] + (dir ? 1 : -1);
        nbl[lc][2 * a + dir] = (a < d && xa >= S.lo[a] && xa < S.hi[a])
                                   ? l + (dir ? bstride[a] : -bstride[a]) : -1;
      }
  }
  __syncthreads();
  // stencil: items (cell, m, trial dof)
  if (want_mat) {
    for (int it = threadIdx.x; it < cc * nm * r; it += blockDim.x) {
      const int lc = it % cc, m = (it / cc) % nm, kp = it / (cc * nm);
      const int x[3] = {cellx[lc][0], cellx[lc][1], cellx[lc][2]};
      double out[8];
      cell_stencil(g, cellg[lc], x, mom, parts, m, kp, out);
      for (int k = 0; k < r; ++k) {
        K(lc, m, 0, k, kp) = out[k];
        K(lc, m, 1, k, kp) = out[r + k];
      }
    }
  }
  __syncthreads();
  // apply: Y = K Phi for every (cell, column)
  for (int p = threadIdx.x; p < cc * ncol; p += blockDim.x) {
    const int lc = p % cc, col = p / cc;
    const int l = c0 + lc;
    double Y[4] = {0.0, 0.0, 0.0, 0.0};
    if (col < NE) {
      const double* cp = phi + S.phi_off + (long long)col * r * nE;
      double ps[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < r; ++k) ps[k] = cp[(long long)k * nE + l];
      if (want_mat) {
        for (int m = 0; m < nm; ++m)
          for (int k = 0; k < r; ++k) {
            double v = 0.0;
            for (int kp = 0; kp < r; ++kp) v += K(lc, m, 0, k, kp) * ps[kp];
            Y[k] += v;
          }
        for (int m = 1; m < nm; ++m) {
          const int ln = nbl[lc][m - 1];
          if (ln < 0) continue;
          double po[4] = {0.0, 0.0, 0.0, 0.0};
          for (int k = 0; k < r; ++k) po[k] = cp[(long long)k * nE + ln];
          for (int k = 0; k < r; ++k) {
            double v = 0.0;
            for (int kp = 0; kp < r; ++kp) v += K(lc, m, 1, k, kp) * po[kp];
            Y[k] += v;
          }
        }
      }
      for (int k = 0; k < r; ++k) Phil[((size_t)lc * r + k) * stride + col] = ps[k];
    } else {
      const int x[3] = {cellx[lc][0], cellx[lc][1], cellx[lc][2]};
      cell_rhs(g, cellg[lc], x, mom, parts, Y);
    }
    for (int k = 0; k < r; ++k) Yl[((size_t)lc * r + k) * stride + col] = Y[k];
  }
  __syncthreads();
  // contract: partial(i, j) = sum over the chunk's rows of Phi(row, i) Y(row, j)
  const int j = threadIdx.x % COLS, grp = threadIdx.x / COLS;
  double acc[COLS];
#pragma unroll
  for (int i = 0; i < COLS; ++i) acc[i] = 0.0;
  if (j < ncol) {
    for (int lc = grp; lc < cc; lc += NG) {
      for (int k = 0; k < r; ++k) {
        const double y = Yl[((size_t)lc * r + k) * stride + j];
        const double* pr = Phil + ((size_t)lc * r + k) * stride;
#pragma unroll
        for (int i = 0; i < COLS; ++i)
          if (i < NE) acc[i] += pr[i] * y;
      }
    }
  }
  __syncthreads();
  // fixed-order tree reduction over the NG groups in the staging area
  double* red = Phil;   // sized for (NG / 2) * COLS * stride doubles (diag_lds_doubles)
#pragma unroll
  for (int half = NG / 2; half >= 1; half /= 2) {
    if (grp >= half && grp < 2 * half && j < ncol) {
#pragma unroll
      for (int i = 0; i < COLS; ++i)
        if (i < NE) red[((size_t)(grp - half) * COLS + i) * stride + j] = acc[i];
    }
    __syncthreads();
    if (grp < half && j < ncol) {
#pragma unroll
      for (int i = 0; i < COLS; ++i)
        if (i < NE) acc[i] += red[((size_t)grp * COLS + i) * stride + j];
    }
    __syncthreads();
  }
  if (grp == 0 && j < ncol) {
    double* out = partial + (long long)blockIdx.x * COLS * stride;
#pragma unroll
    for (int i = 0; i < COLS; ++i)
      if (i < NE) out[i * stride + j] = acc[i];
  }
}

// Sum the chunk partials of every box in chunk order; write A[E][E] and f_E.
template <int COLS>
__global__ __launch_bounds__(256) void k_reduce_diag(const Sub* __restrict__ subs,
                                                     const int* __restrict__ first_chunk,
                                                     const double* __restrict__ partial,
                                                     int has_mat, int has_rhs,
                                                     double* __restrict__ blocks,
                                                     double* __restrict__ fN) {
  constexpr int stride = COLS + 1;
  const Sub S = subs[blockIdx.x];
  const int q0 = first_chunk[blockIdx.x], q1 = first_chunk[blockIdx.x + 1];
  const int NE = S.NE, ncol = NE + (has_rhs ? 1 : 0);
  for (int idx = threadIdx.x; idx < NE * ncol; idx += blockDim.x) {
    const int i = idx / ncol, jj = idx % ncol;
    double v = 0.0;
    for (int q = q0; q < q1; ++q) v += partial[(long long)q * COLS * stride + i * stride + jj];
    if (jj < NE) {
      if (has_mat) blocks[S.blk_off + (long long)i * NE + jj] = v;
    } else {
      fN[S.pn_off + i] = v;
    }
  }
}

// Coupling block A[lo][hi] of one coarse interface: one workgroup per interface.
template <int COLS>
__global__ __launch_bounds__(256) void k_assemble_iface(Geom g, const Sub* __restrict__ subs,
                                                        const Iface* __restrict__ ifs,
                                                        const double* __restrict__ phi,
                                                        const double* __restrict__ mom,
                                                        int parts, double* __restrict__ blocks,
                                                        int chunk) {
  extern __shared__ double lds[];
  const Iface I = ifs[blockIdx.x];
  const Sub SL = subs[I.lo], SH = subs[I.hi];
  const int a = I.axis, r = g.r, d = g.dim;
  const int NL = SL.NE, NH = SH.NE;
  constexpr int stride = COLS + 1;
  constexpr int NG = 256 / COLS;
  double* Phil = lds;
  double* Yl = lds + (size_t)chunk * r * stride;
  int tax[2] = {0, 0}, nt = 0;
  for (int b = 0; b < d; ++b)
    if (b != a) tax[nt++] = b;
  const int ext0 = SL.hi[tax[0]] - SL.lo[tax[0]];
  const int ncolmax = max(NL, NH);
  const bool gam = parts & PART_GAMMA, pen = parts & PART_PEN;
  const int j = threadIdx.x % COLS, grp = threadIdx.x / COLS;
  const int bxL = SL.hi[0] - SL.lo[0], byL = SL.hi[1] - SL.lo[1];
  const int bxH = SH.hi[0] - SH.lo[0], byH = SH.hi[1] - SH.lo[1];
  double acc[COLS];
#pragma unroll
  for (int i = 0; i < COLS; ++i) acc[i] = 0.0;
  for (int q0 = 0; q0 < I.nf; q0 += chunk) {
    const int cc = min(chunk, I.nf - q0);
    for (int p = threadIdx.x; p < cc * ncolmax; p += 256) {
      const int lq = p % cc, col = p / cc;
      const int q = q0 + lq;
      int x0[3] = {0, 0, 0}, x1[3];
      x0[a] = SL.hi[a] - 1;
      x0[tax[0]] = SL.lo[tax[0]] + (nt > 0 ? q % ext0 : 0);
      if (nt > 1) x0[tax[1]] = SL.lo[tax[1]] + q / ext0;
      for (int b = 0; b < 3; ++b) x1[b] = x0[b];
      x1[a] = SH.lo[a];
      const int l0 = (x0[0] - SL.lo[0]) + bxL * ((x0[1] - SL.lo[1]) + byL * (x0[2] - SL.lo[2]));
      const int l1 = (x1[0] - SH.lo[0]) + bxH * ((x1[1] - SH.lo[1]) + byH * (x1[2] - SH.lo[2]));
      const int e0 = cell_index(g, x0), e1 = cell_index(g, x1);
      if (col < NH) {
        const double* cp = phi + SH.phi_off + (long long)col * r * SH.nE;
        double ps[4] = {0.0, 0.0, 0.0, 0.0}, po[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < r; ++k) po[k] = cp[(long long)k * SH.nE + l1];
        FaceCtx f;
        f.a = a;
        f.alpha = 1.0;
        f.interior = true;
        f.ks = g.perm[e0];
        f.ko = g.perm[e1];
        load_moments(g, mom, e0, a, 1, f.ms);
        load_moments(g, mom, e1, a, 0, f.mo);
        double Y[4] = {0.0, 0.0, 0.0, 0.0};
        face_rows(g, f, ps, po, gam, pen, Y);
        for (int k = 0; k < r; ++k) Yl[(lq * r + k) * stride + col] = Y[k];
      }
      if (col < NL) {
        const double* cp = phi + SL.phi_off + (long long)col * r * SL.nE;
        for (int k = 0; k < r; ++k) Phil[(lq * r + k) * stride + col] = cp[(long long)k * SL.nE + l0];
      }
    }
    __syncthreads();
    if (j < NH) {
      for (int lq = grp; lq < cc; lq += NG) {
        for (int k = 0; k < r; ++k) {
          const double y = Yl[(lq * r + k) * stride + j];
          const double* pr = Phil + (lq * r + k) * stride;
#pragma unroll
          for (int i = 0; i < COLS; ++i)
            if (i < NL) acc[i] += pr[i] * y;
        }
      }
    }
    __syncthreads();
  }
  double* red = lds;
  if (j < NH) {
#pragma unroll
    for (int i = 0; i < COLS; ++i)
      if (i < NL) red[(grp * COLS + i) * stride + j] = acc[i];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NL * NH; idx += 256) {
    const int i = idx / NH, jj = idx % NH;
    double v = 0.0;
    for (int q = 0; q < NG; ++q) v += red[(q * COLS + i) * stride + jj];
    blocks[I.blk_off + (long long)i * NH + jj] = v;
  }
}

template <int COLS>
static hipError_t launch_assemble_t(const AsmLayout& L, const Geom& g, const Sub* d_subs,
                                    int n_sub, const Iface* d_ifaces, int n_iface,
                                    const double* phi, const double* mom, int parts,
                                    double* blocks, double* fN, hipStream_t st) {
  const bool has_mat = (parts & (PART_GAMMA | PART_PEN)) && blocks;
  const bool has_rhs = (parts & (PART_RHS_CONST | PART_RHS_GAMMA)) && fN;
  const int pdiag = (has_mat ? (PART_GAMMA | PART_PEN) & parts : 0) |
                    (has_rhs ? (PART_RHS_CONST | PART_RHS_GAMMA) & parts : 0);
  if (n_sub > 0 && pdiag) {
    const size_t lds = sizeof(double) * diag_lds_doubles(COLS, g.r, g.dim);
    ktimer_begin(KK_ASM_DIAG, st);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_assemble_diag<COLS>), dim3(L.n_chunks), dim3(256), lds,
                       st, g, d_subs, L.chunks, phi, mom, pdiag, L.partial);
    ktimer_end(-1.0, -1.0, st);
    ktimer_begin(KK_ASM_REDUCE, st);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reduce_diag<COLS>), dim3(n_sub), dim3(256), 0, st,
                       d_subs, L.first_chunk, L.partial, has_mat ? 1 : 0, has_rhs ? 1 : 0, blocks,
                       fN);
    ktimer_end(-1.0, -1.0, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_iface > 0 && has_mat) {
    constexpr int stride = COLS + 1;
    const size_t budget = 72 * 1024;
    int chunk = (int)(budget / (sizeof(double) * 2 * g.r * stride));
    if (chunk < 1) chunk = 1;
    const size_t lds_chunk = sizeof(double) * 2 * (size_t)chunk * g.r * stride;
    const size_t lds_red = sizeof(double) * (size_t)(256 / COLS) * COLS * stride;
    const size_t lds = lds_chunk > lds_red ? lds_chunk : lds_red;
    ktimer_begin(KK_ASM_IFACE, st);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_assemble_iface<COLS>), dim3(n_iface), dim3(256), lds,
                       st, g, d_subs, d_ifaces, phi, mom, parts, blocks, chunk);
    ktimer_end(-1.0, -1.0, st);
    return hipGetLastError();
  }
  return hipSuccess;
}

int assemble_cols(int max_ne) { return max_ne + 1 <= 16 ? 16 : (max_ne + 1 <= 32 ? 32 : 64); }

hipError_t assemble_prepare(const Geom& g, const std::vector<Sub>& subs, int max_ne,
                            AsmLayout& L, long long& bytes) {
  std::vector<int> chunks, first(1, 0);
  const int ch = assemble_cols(max_ne) <= 32 ? kChunk : kChunk / 2;
  for (size_t s = 0; s < subs.size(); ++s) {
    for (int c0 = 0; c0 < subs[s].nE; c0 += ch) {
      chunks.push_back((int)s);
      chunks.push_back(c0);
    }
    first.push_back((int)chunks.size() / 2);
  }
  L.n_chunks = (int)chunks.size() / 2;
  const int cols = assemble_cols(max_ne);
  hipError_t e;
  if ((e = hipMalloc(&L.chunks, chunks.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMemcpy(L.chunks, chunks.data(), chunks.size() * sizeof(int),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  if ((e = hipMalloc(&L.first_chunk, first.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMemcpy(L.first_chunk, first.data(), first.size() * sizeof(int),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  const size_t np = (size_t)L.n_chunks * cols * (cols + 1);
  if ((e = hipMalloc(&L.partial, np * sizeof(double))) != hipSuccess) return e;
  bytes += (long long)(np * sizeof(double) + (chunks.size() + first.size()) * sizeof(int));
  // the interface kernel may use more than 64 KB of dynamic LDS
  const int stride = cols + 1;
  const size_t budget = 72 * 1024;
  int chunk = (int)(budget / (sizeof(double) * 2 * g.r * stride));
  if (chunk < 1) chunk = 1;
  size_t lds = std::max(sizeof(double) * 2 * (size_t)chunk * g.r * stride,
                        sizeof(double) * (size_t)(256 / cols) * cols * stride);
  const int dl = (int)(sizeof(double) * diag_lds_doubles(cols, g.r, g.dim));
  if (cols == 16)
    e = hipFuncSetAttribute((const void*)k_assemble_diag<16>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, dl);
  else if (cols == 32)
    e = hipFuncSetAttribute((const void*)k_assemble_diag<32>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, dl);
  else
    e = hipFuncSetAttribute((const void*)k_assemble_diag<64>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, dl);
  if (e != hipSuccess) return e;
  if (cols == 16)
    e = hipFuncSetAttribute((const void*)k_assemble_iface<16>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  else if (cols == 32)
    e = hipFuncSetAttribute((const void*)k_assemble_iface<32>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  else
    e = hipFuncSetAttribute((const void*)k_assemble_iface<64>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return e;
}

void assemble_free(AsmLayout& L) {
  if (L.chunks) (void)hipFree(L.chunks);
  if (L.first_chunk) (void)hipFree(L.first_chunk);
  if (L.partial) (void)hipFree(L.partial);
  L = AsmLayout{};
}

hipError_t launch_assemble(const AsmLayout& L, const Geom& g, const Sub* d_subs, int n_sub,
                           int max_ne, const Iface* d_ifaces, int n_iface, const double* phi,
                           const double* mom, int parts, double* blocks, double* fN,
                           hipStream_t st) {
  const int cols = assemble_cols(max_ne);
  if (cols == 16)
    return launch_assemble_t<16>(L, g, d_subs, n_sub, d_ifaces, n_iface, phi, mom, parts, blocks,
                                 fN, st);
  if (cols == 32)
    return launch_assemble_t<32>(L, g, d_subs, n_sub, d_ifaces, n_iface, phi, mom, parts, blocks,
                                 fN, st);
  return launch_assemble_t<64>(L, g, d_subs, n_sub, d_ifaces, n_iface, phi, mom, parts, blocks,
                               fN, st);
}

// ---------------------------------------------------------------------------
// eq. reducedSystem: out = base + sum_q theta_q terms[q] (q in increasing order).
__global__ __launch_bounds__(256) void k_affine_sum(const double* __restrict__ base,
                                                    const double* __restrict__ terms, long long n,
                                                    const double* __restrict__ theta, int nq,
                                                    double* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double v = base[i];
    for (int q = 0; q < nq; ++q) v = v + theta[q] * terms[(long long)q * n + i];
    out[i] = v;
  }
}

hipError_t launch_affine_sum(const double* base, const double* terms, long long n,
                             const double* theta, int nq, double* out, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  ktimer_begin(KK_AFFINE_SUM, st);
  hipLaunchKernelGGL(k_affine_sum, dim3((unsigned)nb), dim3(256), 0, st, base, terms, n, theta,
                     nq, out);
  ktimer_end(2.0 * (double)n * nq, 8.0 * (double)n * (nq + 2), st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// eq. leastSquaresFit: r_q = (Lambda^q, Pi lambda(s))_{L2} with the P1
// projection Pi lambda(s) evaluated by the 2-point Gauss rule; theta solves
// G theta = r with the Cholesky factor of the profile Gram matrix G.
__global__ __launch_bounds__(256) void k_lsq_partial(Geom g, const double* __restrict__ sat,
                                                     const double* __restrict__ prof, int nprof,
                                                     double* __restrict__ partial) {
  __shared__ double red[256];
  const int nc = g.ncell, d = g.dim, r = g.r;
  double lp[4];  // P1 projection coefficients of lambda(s) on this thread's cell
  double acc[kMaxProfiles];
  for (int q = 0; q < nprof; ++q) acc[q] = 0.0;
  const double gp = 1.0 / kSqrt3;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    double co[4] = {0, 0, 0, 0};
    for (int k = 0; k < r; ++k) co[k] = sat[(long long)k * nc + c];
    for (int k = 0; k < r; ++k) lp[k] = 0.0;
    const int nq = 1 << d;
    const double w = g.vol / nq;
    for (int p = 0; p < nq; ++p) {
      double sq[3];
      double v = co[0];
      for (int a = 0; a < d; ++a) {
        sq[a] = kSqrt3 * (((p >> a) & 1) ? gp : -gp);
        v += sq[a] * co[a + 1];
      }
      const double lam = total_mobility(g, v * g.isv) * w;
      lp[0] += lam * g.isv;
      for (int a = 0; a < d; ++a) lp[a + 1] += lam * sq[a] * g.isv;
    }
    for (int q = 0; q < nprof; ++q) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s += prof[(long long)q * r * nc + (long long)k * nc + c] * lp[k];
      acc[q] += s;
    }
  }
  for (int q = 0; q < nprof; ++q) {
    red[threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long long)blockIdx.x * nprof + q] = red[0];
    __syncthreads();
  }
}

__global__ void k_lsq_final(const double* __restrict__ partial, int nblocks, int nprof,
                            const double* __restrict__ L, double* __restrict__ theta) {
  __shared__ double rhs[kMaxProfiles];
  const int q = threadIdx.x;
  if (q < nprof) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += partial[(long long)b * nprof + q];
    rhs[q] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // forward then backward substitution with the lower Cholesky factor L
    double y[kMaxProfiles];
    for (int i = 0; i < nprof; ++i) {
      double v = rhs[i];
      for (int k = 0; k < i; ++k) v -= L[i * nprof + k] * y[k];
      y[i] = v / L[i * nprof + i];
    }
    for (int i = nprof - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < nprof; ++k) v -= L[k * nprof + i] * y[k];
      y[i] = v / L[i * nprof + i];
    }
    for (int i = 0; i < nprof; ++i) theta[i] = y[i];
  }
}

hipError_t launch_lsq(const Geom& g, const double* sat, const double* prof, int nprof,
                      const double* gchol, double* partial, int nblocks, double* theta,
                      hipStream_t st) {
  ktimer_begin(KK_LSQ, st);
  hipLaunchKernelGGL(k_lsq_partial, dim3(nblocks), dim3(256), 0, st, g, sat, prof, nprof,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lsq_final, dim3(1), dim3(64), 0, st, partial, nblocks, nprof, gchol, theta);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

}  // namespace lrbms
